"""The seeded input generator against the oracle: the separable load vectors
it produces equal the oracle's general space-time quadrature."""
import numpy as np
import pytest

import synth
from oracle import fem, problems


@pytest.mark.parametrize("p", [1, 2])
def test_manufactured_load_vector_matches_oracle_quadrature(p):
    wl = synth.Workload("t", 8, 1.0, 6, p, 4 * np.pi)
    nodes = synth.uniform_nodes(wl.T, wl.N_t)
    Fs = synth.manufactured_rhs(wl, nodes, homogenised=False)
    prob = problems.OmegaSolution(wl.omega)
    Fo = fem.load_vector(prob.f, wl.n, nodes, p, m_space=6, m_time=8)[1:]
    assert np.abs(Fs - Fo).max() < 1e-12 * np.abs(Fo).max()


def test_homogenised_load_is_load_of_f_hat():
    wl = synth.Workload("t", 6, 1.0, 4, 1, np.pi)
    nodes = synth.uniform_nodes(wl.T, wl.N_t)
    Fs = synth.manufactured_rhs(wl, nodes, homogenised=True)
    prob = problems.OmegaSolution(wl.omega)
    fhat = lambda x, y, t: prob.f(x, y, t) - 2 * np.pi ** 2 * prob.psi0(x, y)
    Fo = fem.load_vector(fhat, wl.n, nodes, 1, m_space=6, m_time=8)[1:]
    assert np.abs(Fs - Fo).max() < 1e-12 * np.abs(Fo).max()


def test_psi_hat_nodal_matches_oracle_interpolant():
    wl = synth.Workload("t", 5, 1.0, 3, 2, np.pi)
    nodes = synth.uniform_nodes(wl.T, wl.N_t)
    prob = problems.OmegaSolution(wl.omega)
    ref = fem.interpolate(lambda x, y, t: prob.psi(x, y, t) - prob.psi0(x, y), wl.n, nodes, 2)[1:]
    assert np.abs(synth.manufactured_psi_hat(wl, nodes) - ref).max() < 1e-14


def test_workload_sizes():
    assert synth.WORKLOADS["c0"].dofs == 3600
    assert synth.WORKLOADS["c1"].n_x == 16129
    assert synth.WORKLOADS["c2"].dofs == 16646400
    assert synth.WORKLOADS["c4"].n_t == 512
    assert synth.WORKLOADS["c4"].dofs == 133693952


def test_random_rhs_is_seeded():
    a = synth.random_rhs(3, 4, 5)
    b = synth.random_rhs(3, 4, 5)
    assert np.array_equal(a, b) and a.dtype == np.complex128
