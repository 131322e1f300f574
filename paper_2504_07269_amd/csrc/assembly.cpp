// Assembly of the temporal and spatial matrices (Sec. 3, eqs. (matrix_t) and
// (matrix_x)) and the library's error plumbing.
#include <cstring>
#include <string>

#include "common.h"

namespace stfem {

static thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}
void clear_error() { g_last_error.clear(); }

}  // namespace stfem

using namespace stfem;

extern "C" const char* stfem_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* stfem_strerror(int s) {
    switch (s) {
        case STFEM_OK: return "ok";
        case STFEM_EINVAL: return "invalid argument";
        case STFEM_ENOMEM: return "out of memory";
        case STFEM_EHIP: return "HIP runtime error";
        case STFEM_ENOTDIAG: return "temporal eigen-decomposition failed";
        case STFEM_ENOCONV: return "refinement did not converge";
        case STFEM_EBREAKDOWN: return "zero or non-finite pivot";
        default: return "unknown status";
    }
}

// Element matrices of continuous Lagrange elements on [t_a, t_a + h] with
// equispaced nodes, local dofs in position order.  Rows are test functions.
// P1: mass h/6 [[2,1],[1,2]];  int phi_b' phi_a = 1/2 [[-1,1],[-1,1]].
// P2: mass h/30 [[4,2,-1],[2,16,2],[-1,2,4]];
//     int phi_b' phi_a = 1/6 [[-3,4,-1],[-4,0,4],[1,-4,3]].
static void time_element(int p, double h, double Me[3][3], double Be[3][3]) {
    if (p == 1) {
        const double m[2][2] = {{2, 1}, {1, 2}}, b[2][2] = {{-1, 1}, {-1, 1}};
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < 2; ++c) {
                Me[a][c] = h * m[a][c] / 6.0;
                Be[a][c] = 0.5 * b[a][c];
            }
    } else {
        const double m[3][3] = {{4, 2, -1}, {2, 16, 2}, {-1, 2, 4}};
        const double b[3][3] = {{-3, 4, -1}, {-4, 0, 4}, {1, -4, 3}};
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                Me[a][c] = h * m[a][c] / 30.0;
                Be[a][c] = b[a][c] / 6.0;
            }
    }
}

extern "C" int assemble_1d_time(int n_el, const double* t_nodes, int p, double* M_t, double* B_t,
                                double* m_col0, double* b_col0) {
    clear_error();
    if (n_el < 1 || !t_nodes || !M_t || !B_t || (p != 1 && p != 2))
        return fail(STFEM_EINVAL, "assemble_1d_time: need n_el >= 1, p in {1,2}, non-null arrays");
    if (t_nodes[0] != 0.0) return fail(STFEM_EINVAL, "assemble_1d_time: t_nodes[0] must be 0");
    for (int e = 0; e < n_el; ++e)
        if (!(t_nodes[e + 1] > t_nodes[e]))
            return fail(STFEM_EINVAL, "assemble_1d_time: nodes must be strictly increasing");
    const int nt = p * n_el;
    std::memset(M_t, 0, sizeof(double) * (size_t)nt * nt);
    std::memset(B_t, 0, sizeof(double) * (size_t)nt * nt);
    if (m_col0) std::memset(m_col0, 0, sizeof(double) * nt);
    if (b_col0) std::memset(b_col0, 0, sizeof(double) * nt);
    double Me[3][3], Be[3][3];
    for (int e = 0; e < n_el; ++e) {
        time_element(p, t_nodes[e + 1] - t_nodes[e], Me, Be);
        for (int a = 0; a <= p; ++a) {
            const int ga = p * e + a - 1;          // dof index without t_0
            if (ga < 0) continue;
            for (int c = 0; c <= p; ++c) {
                const int gc = p * e + c - 1;
                if (gc < 0) {                      // coupling to the removed t_0 dof
                    if (m_col0) m_col0[ga] += Me[a][c];
                    if (b_col0) b_col0[ga] += Be[a][c];
                    continue;
                }
                M_t[(size_t)ga * nt + gc] += Me[a][c];
                B_t[(size_t)ga * nt + gc] += Be[a][c];
            }
        }
    }
    return STFEM_OK;
}

// The right-diagonal mesh: every cell [x_i, x_i+h] x [y_j, y_j+h] is cut into
// the triangles (SW, SE, NE) and (SW, NE, NW).  The stencil of an interior
// vertex is assembled from the six triangles around it: P1 element mass
// |T|/12 (1 + delta_ab) and stiffness |T| grad(phi_a).grad(phi_b).
extern "C" int assemble_2d_space(int n, double* M_stencil, double* A_stencil, int* n_x, int* kd) {
    clear_error();
    if (n < 2 || !M_stencil || !A_stencil)
        return fail(STFEM_EINVAL, "assemble_2d_space: need n >= 2 and non-null stencil arrays");
    const double h = 1.0 / n;
    // neighbour offsets in STFEM_ST_* order
    const int off[7][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}};
    double Mst[7] = {0}, Ast[7] = {0};
    // Triangles with a vertex at the origin, in units of h: the origin's cell
    // and its west, south and south-west neighbour cells.
    for (int ci = -1; ci <= 0; ++ci)
        for (int cj = -1; cj <= 0; ++cj) {
            const int tri[2][3][2] = {{{ci, cj}, {ci + 1, cj}, {ci + 1, cj + 1}},
                                      {{ci, cj}, {ci + 1, cj + 1}, {ci, cj + 1}}};
            for (int t = 0; t < 2; ++t) {
                int at = -1;
                for (int a = 0; a < 3; ++a)
                    if (tri[t][a][0] == 0 && tri[t][a][1] == 0) at = a;
                if (at < 0) continue;
                // P1 gradients: grad phi_a = rot(P_{a+2} - P_{a+1}) / (2|T|) for a
                // counter-clockwise triangle
                double px[3], py[3];
                for (int a = 0; a < 3; ++a) { px[a] = tri[t][a][0] * h; py[a] = tri[t][a][1] * h; }
                const double area2 = (px[1] - px[0]) * (py[2] - py[0]) - (px[2] - px[0]) * (py[1] - py[0]);
                double gx[3], gy[3];
                for (int a = 0; a < 3; ++a) {
                    const int b = (a + 1) % 3, c = (a + 2) % 3;
                    gx[a] = (py[b] - py[c]) / area2;
                    gy[a] = (px[c] - px[b]) / area2;
                }
                const double area = 0.5 * area2;
                for (int b = 0; b < 3; ++b) {
                    const int dx = tri[t][b][0], dy = tri[t][b][1];
                    int s = -1;
                    for (int q = 0; q < 7; ++q)
                        if (off[q][0] == dx && off[q][1] == dy) s = q;
                    if (s < 0) return fail(STFEM_EINVAL, "assemble_2d_space: internal stencil error");
                    Mst[s] += area / 12.0 * (b == at ? 2.0 : 1.0);
                    Ast[s] += area * (gx[at] * gx[b] + gy[at] * gy[b]);
                }
            }
        }
    for (int q = 0; q < 7; ++q) {
        M_stencil[q] = Mst[q];
        A_stencil[q] = std::fabs(Ast[q]) < 1e-14 ? 0.0 : Ast[q];
    }
    if (n_x) *n_x = (n - 1) * (n - 1);
    if (kd) *kd = n;
    return STFEM_OK;
}
