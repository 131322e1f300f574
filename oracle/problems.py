"""Manufactured solutions of i d_t psi - Lap_x psi = f on (0,1)^2 x (0,T) with
homogeneous Dirichlet data (Sec. 1, eq. (SchroedingerBeschraenkt)); test
infrastructure only.

Each problem provides psi, d_t psi, grad_x psi, the right-hand side f derived
by hand from f = i d_t psi - Lap psi, and psi_0 = psi(., 0).
"""
import numpy as np

PI = np.pi


class PaperSolution:
    """psi = e^{it} sin(pi x) sin(pi y) sin(t x y), psi_0 = 0 (Sec. 4)."""

    name = "paper"

    def psi(self, x, y, t):
        return np.exp(1j * t) * np.sin(PI * x) * np.sin(PI * y) * np.sin(t * x * y)

    def dt(self, x, y, t):
        s = np.sin(PI * x) * np.sin(PI * y)
        return np.exp(1j * t) * s * (1j * np.sin(t * x * y) + x * y * np.cos(t * x * y))

    def grad(self, x, y, t):
        e = np.exp(1j * t)
        g = np.sin(t * x * y)
        c = np.cos(t * x * y)
        s = np.sin(PI * x) * np.sin(PI * y)
        gx = e * (PI * np.cos(PI * x) * np.sin(PI * y) * g + s * c * t * y)
        gy = e * (PI * np.sin(PI * x) * np.cos(PI * y) * g + s * c * t * x)
        return gx, gy

    def f(self, x, y, t):
        e = np.exp(1j * t)
        g = np.sin(t * x * y)
        c = np.cos(t * x * y)
        s = np.sin(PI * x) * np.sin(PI * y)
        mixed = y * np.cos(PI * x) * np.sin(PI * y) + x * np.sin(PI * x) * np.cos(PI * y)
        return e * (s * g * (2 * PI ** 2 - 1 + t ** 2 * (x ** 2 + y ** 2))
                    + 1j * x * y * c * s - 2 * PI * t * c * mixed)

    def psi0(self, x, y):
        return np.zeros_like(x, dtype=np.complex128)


class OmegaSolution:
    """psi = sin(pi x) sin(pi y) (1 + t^2) e^{i omega t}, psi_0 = sin(pi x) sin(pi y)."""

    name = "omega"

    def __init__(self, omega):
        self.omega = float(omega)

    def psi(self, x, y, t):
        return np.sin(PI * x) * np.sin(PI * y) * (1 + t ** 2) * np.exp(1j * self.omega * t)

    def dt(self, x, y, t):
        w = self.omega
        return np.sin(PI * x) * np.sin(PI * y) * np.exp(1j * w * t) * (2 * t + 1j * w * (1 + t ** 2))

    def grad(self, x, y, t):
        a = (1 + t ** 2) * np.exp(1j * self.omega * t)
        return (a * PI * np.cos(PI * x) * np.sin(PI * y), a * PI * np.sin(PI * x) * np.cos(PI * y))

    def f(self, x, y, t):
        w = self.omega
        s = np.sin(PI * x) * np.sin(PI * y)
        return s * np.exp(1j * w * t) * (2 * PI ** 2 * (1 + t ** 2) - w * (1 + t ** 2) + 2j * t)

    def psi0(self, x, y):
        return (np.sin(PI * x) * np.sin(PI * y)).astype(np.complex128)
