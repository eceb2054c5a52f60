// Principal permeabilities, principal axes and material class of a
// permeability tensor (§2: spectral form eq. 3dK_eigen and the three classes
// listed after it; App. C for averaging the off-diagonals; §6.4 for the
// reduced two-dimensional evaluation).  Host code: nine numbers in, no GPU.
#include <cmath>
#include <cstring>

#include "porestokes.h"

namespace {

bool finite9(const double *k)
{
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(k[i])) return false;
    return true;
}

// Cyclic Jacobi method on a symmetric 3x3 matrix A: each plane rotation J in
// the (p, q) plane, A <- J^T A J, makes A[p][q] zero; V <- V J accumulates
// them, so that on return A_in = V diag(A) V^T with V orthogonal.  The angle
// of the rotation satisfies cot(2 phi) = (A_qq - A_pp) / (2 A_pq), and its
// tangent is taken as the root of smaller magnitude of t^2 + 2 t cot(2 phi) - 1 = 0.
void jacobi3(double A[3][3], double V[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    static const int P[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int sweep = 0; sweep < 64; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off == 0.0 || off <= 1e-36 * dia) break;
        for (const auto &pq : P) {
            const int p = pq[0], q = pq[1];
            if (A[p][q] == 0.0) continue;
            const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
            double t;
            if (std::fabs(theta) > 1e150) t = 0.5 / theta;
            else t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
            const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
            double J[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
            J[p][p] = c;
            J[q][q] = c;
            J[p][q] = s;
            J[q][p] = -s;
            double AJ[3][3], B[3][3], VJ[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    AJ[i][j] = A[i][0] * J[0][j] + A[i][1] * J[1][j] + A[i][2] * J[2][j];
                    VJ[i][j] = V[i][0] * J[0][j] + V[i][1] * J[1][j] + V[i][2] * J[2][j];
                }
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) B[i][j] = J[0][i] * AJ[0][j] + J[1][i] * AJ[1][j] + J[2][i] * AJ[2][j];
            // the annihilated pair is zero by construction; keep A exactly symmetric
            B[p][q] = B[q][p] = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    A[i][j] = (i == j) ? B[i][j] : 0.5 * (B[i][j] + B[j][i]);
                    V[i][j] = VJ[i][j];
                }
        }
    }
}

bool same(double a, double b, double tol) { return std::fabs(a - b) <= tol * std::fmax(std::fabs(a), std::fabs(b)); }

double rel_gap(double a, double b)
{
    const double m = std::fmax(std::fabs(a), std::fabs(b));
    return m > 0.0 ? std::fabs(a - b) / m : 0.0;
}

}  // namespace

extern "C" {

pm_status pm_principal_axes(const double k[9], double rel_tol, pm_principal *out)
{
    if (!k || !out || !std::isfinite(rel_tol) || rel_tol < 0.0 || !finite9(k)) return PM_ERR_ARG;
    std::memset(out, 0, sizeof *out);
    double A[3][3], V[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            out->k_sym[i * 3 + j] = 0.5 * (k[i * 3 + j] + k[j * 3 + i]);
            A[i][j] = out->k_sym[i * 3 + j];
        }
    jacobi3(A, V);
    // ascending order of the principal values, columns of V with them
    int ord[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (A[ord[j]][ord[j]] < A[ord[i]][ord[i]]) {
                const int t = ord[i];
                ord[i] = ord[j];
                ord[j] = t;
            }
    double col[3][3];
    for (int c = 0; c < 3; ++c) {
        out->lambda[c] = A[ord[c]][ord[c]];
        for (int r = 0; r < 3; ++r) col[c][r] = V[r][ord[c]];
    }
    // columns 0 and 1: largest-magnitude component positive; column 2 = col0 x col1
    for (int c = 0; c < 2; ++c) {
        int m = 0;
        for (int r = 1; r < 3; ++r)
            if (std::fabs(col[c][r]) > std::fabs(col[c][m])) m = r;
        if (col[c][m] < 0.0)
            for (int r = 0; r < 3; ++r) col[c][r] = -col[c][r];
    }
    col[2][0] = col[0][1] * col[1][2] - col[0][2] * col[1][1];
    col[2][1] = col[0][2] * col[1][0] - col[0][0] * col[1][2];
    col[2][2] = col[0][0] * col[1][1] - col[0][1] * col[1][0];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) out->R[r * 3 + c] = col[c][r];
    // material class (§2)
    const double *l = out->lambda;
    out->distinct = -1;
    if (same(l[0], l[2], rel_tol)) {
        out->cls = PM_ISOTROPIC;
    } else {
        const bool e01 = same(l[0], l[1], rel_tol), e12 = same(l[1], l[2], rel_tol);
        if (e01 || e12) {
            out->cls = PM_TRANSVERSE;
            const bool low_pair = e01 && (!e12 || rel_gap(l[0], l[1]) <= rel_gap(l[1], l[2]));
            out->distinct = low_pair ? 2 : 0;
        } else {
            out->cls = PM_ORTHOTROPIC;
        }
    }
    out->ratio = l[0] > 0.0 ? l[2] / l[0] : INFINITY;
    return PM_OK;
}

pm_status pm_plane_angle(const double k[9], int a, int b, double *phi, double lam[2])
{
    if (!k || !phi || !lam || a < 0 || a > 2 || b < 0 || b > 2 || a == b || !finite9(k)) return PM_ERR_ARG;
    const double kaa = k[a * 3 + a], kbb = k[b * 3 + b];
    const double s = 0.5 * (k[a * 3 + b] + k[b * 3 + a]);
    *phi = 0.5 * std::atan2(2.0 * s, kbb - kaa);
    const double m = 0.5 * (kaa + kbb), r = std::hypot(0.5 * (kbb - kaa), s);
    lam[0] = m - r;
    lam[1] = m + r;
    return PM_OK;
}

}  // extern "C"
