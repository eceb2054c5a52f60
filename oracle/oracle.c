/*
 * oracle.c -- plain FP64 CPU reference for the pseudo-unsteady Stokes
 * permeability method (POREMAPS, arXiv 2407.19868).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file: it is used by the test suite, by the smoke check and by
 * the benchmark's CPU-baseline leg.  It shares no code, header or table with
 * the GPU library.
 *
 * It is written for checking by eye against the paper, not for speed:
 *   - staggered MAC grid (§4 "Grid"): u, v, w on the x-, y-, z-faces, p at
 *     cell centres; u(c) is the face between cells c - e_x and c;
 *   - face solid iff either adjacent voxel is solid (no penetration, §4);
 *   - perpendicular second derivatives from the eight neighbourhood cases of
 *     App. B (cases 1-6 for periodic domains; 7 and 8 are only used for
 *     non-periodic outer walls and appear here as stencils only);
 *   - along the component's own axis the standard 3-point stencil, a solid
 *     neighbour face holding an exact zero;
 *   - pseudo-time step of the nondimensional artificial-compressibility
 *     equations (§3, App. A): velocity first (all components from the old
 *     state), then pressure from the new velocity (Algorithm 1 order);
 *   - drive: p = p~ - G x_axis with p~ periodic, i.e. a constant source G on
 *     the momentum equation of the load-axis component (§4 "Simulation
 *     parametrization": initial gradient 1/vx, Re = 0.01, c*^2 = 1.5e6);
 *   - Darcy (§4 eq. darcy, App. C): k_{i,axis} = dx^2 q_i / (Re G), q_i the
 *     mean of u_i over all i-faces;
 *   - optional fixed pressure in the main flow direction (§4, boundary of the
 *     numerically considered domain; Fig. 2 p_in / p_out): p~ held on the
 *     cell layer x_axis = 0, so that p = p_in there and p_out = p_in - G n
 *     one period later; that layer's mass balance is not imposed and it is
 *     left out of the residual's divergence sum.
 *
 * Floating point: FP64, terms summed in the written order (x, then y, then
 * z), built without fast-math or FMA contraction.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct {
    double re;          /* Reynolds number (nu = 1/re)                  */
    double c2;          /* artificial compressibility c*^2              */
    double dt;          /* pseudo-time step                             */
    double tol;         /* stop when r < tol                            */
    double drive;       /* G, nondimensional pressure gradient          */
    double voxel_size;  /* dx, scales k to physical units               */
    int64_t max_sweeps;
    int32_t check_every;
    int32_t warm_start; /* 1: start from the given fields               */
    int32_t stop_rule;  /* 0: residual r, 1: relative flux change eps_q */
    int32_t fixed_pressure; /* 1: §4 fixes the pressure along the drive, read
                           as: p~ is held at its value (0 from rest) on the
                           cell layer x_axis = 0, whose mass balance is not
                           imposed; the velocity stays periodic (§4 keeps the
                           local flux periodic)                             */
} orc_params;

enum { ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_OOM = 2, ORC_NOT_CONVERGED = 4, ORC_DIVERGED = 5,
       ORC_NO_FLOW = 6 };

static int64_t wrap(int64_t i, int64_t n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

typedef struct {
    int64_t n[3]; /* nx, ny, nz */
} grid;

static int64_t at(const grid *g, int64_t x, int64_t y, int64_t z)
{
    return (wrap(z, g->n[2]) * g->n[1] + wrap(y, g->n[1])) * g->n[0] + wrap(x, g->n[0]);
}

/* index of cell c + d e_axis, c given by coordinates */
static int64_t shifted(const grid *g, const int64_t c[3], int axis, int64_t d)
{
    int64_t p[3] = {c[0], c[1], c[2]};
    p[axis] += d;
    return at(g, p[0], p[1], p[2]);
}

/* ------------------------------------------------------------------ flags */

/* FS_k(c) = S(c) or S(c - e_k), for k = x, y, z.  fs is [3][nz][ny][nx]. */
void orc_face_solid(const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz, uint8_t *fs)
{
    grid g = {{nx, ny, nz}};
    const int64_t N = nx * ny * nz;
    for (int k = 0; k < 3; ++k)
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    int64_t c[3] = {x, y, z};
                    int64_t self = at(&g, x, y, z);
                    int64_t back = shifted(&g, c, k, -1);
                    fs[k * N + self] = (mask[self] != 0) || (mask[back] != 0);
                }
}

/* Bit-packed face flags: bits[k][z][y][w], bit b of word w is x = 32 w + b. */
void orc_pack_bits(const uint8_t *fs, int64_t nx, int64_t ny, int64_t nz, uint32_t *bits)
{
    const int64_t N = nx * ny * nz, W = (nx + 31) / 32;
    memset(bits, 0, sizeof(uint32_t) * 3 * (size_t)(W * ny * nz));
    for (int k = 0; k < 3; ++k)
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x)
                    if (fs[k * N + (z * ny + y) * nx + x])
                        bits[((k * nz + z) * ny + y) * W + x / 32] |= (uint32_t)1 << (x % 32);
}

/* -------------------------------------------------------- neighbourhood cases
 *
 * For a fluid face and a perpendicular axis, s_m2, s_m1, s_p1, s_p2 are the
 * solid flags of the same-component faces at offsets -2, -1, +1, +2.  A solid
 * face at offset +-1 puts a wall half a voxel away; a solid face at +-2 (with
 * +-1 fluid) puts it 3/2 voxels away.
 *   case 1: walls on both sides                       (App. B case 1)
 *   case 2: wall at -1/2, fluid at +1, wall at +3/2   (case 2)
 *   case 3: mirror of case 2                          (case 3)
 *   case 4: wall at -1/2, fluid at +1 and +2          (case 4)
 *   case 5: mirror of case 4                          (case 5)
 *   case 6: fluid on both sides                       (case 6)
 */
int orc_case(int s_m2, int s_m1, int s_p1, int s_p2)
{
    if (s_m1 && s_p1) return 1;
    if (s_m1) return s_p2 ? 2 : 4;
    if (s_p1) return s_m2 ? 3 : 5;
    return 6;
}

/* App. B: d2v/dx_i^2 at the face from the values at offsets -2..+2 (grid step 1). */
double orc_d2(int cse, double vm2, double vm1, double v0, double vp1, double vp2)
{
    switch (cse) {
    case 1: return -8.0 * v0;
    case 2: return (8.0 / 3.0) * vp1 - (16.0 / 3.0) * v0;
    case 3: return (8.0 / 3.0) * vm1 - (16.0 / 3.0) * v0;
    case 4: return 2.0 * vp1 - 5.0 * v0 - (1.0 / 5.0) * vp2;
    case 5: return 2.0 * vm1 - (1.0 / 5.0) * vm2 - 5.0 * v0;
    case 6: return vm1 - 2.0 * v0 + vp1;
    case 7: return (4.0 / 3.0) * vp1 - 4.0 * v0;
    case 8: return (4.0 / 3.0) * vm1 - 4.0 * v0;
    default: return NAN;
    }
}

/* ------------------------------------------------------ momentum and mass */

/* Value of component k at face index id; a solid face holds an exact zero. */
static double face_val(const uint8_t *fs, const double *vk, int64_t N, int k, int64_t id)
{
    return fs[k * N + id] ? 0.0 : vk[id];
}

/*
 * Momentum right-hand side at the fluid k-face of cell c for the state (v, p):
 *   F = nu (d2/dx^2 + d2/dy^2 + d2/dz^2) v_k - (p(c) - p(c - e_k)) + G [k == axis]
 */
static double momentum(const grid *g, const uint8_t *fs, const double *const v[3], const double *p,
                       int k, const int64_t c[3], int axis, double nu, double G)
{
    const int64_t N = g->n[0] * g->n[1] * g->n[2];
    const int64_t self = at(g, c[0], c[1], c[2]);
    const double v0 = v[k][self];
    double lap = 0.0;
    for (int i = 0; i < 3; ++i) {
        if (i == k) {
            double vm = face_val(fs, v[k], N, k, shifted(g, c, i, -1));
            double vp = face_val(fs, v[k], N, k, shifted(g, c, i, +1));
            lap += vm - 2.0 * v0 + vp;
        } else {
            int64_t im2 = shifted(g, c, i, -2), im1 = shifted(g, c, i, -1);
            int64_t ip1 = shifted(g, c, i, +1), ip2 = shifted(g, c, i, +2);
            int cse = orc_case(fs[k * N + im2], fs[k * N + im1], fs[k * N + ip1], fs[k * N + ip2]);
            lap += orc_d2(cse, face_val(fs, v[k], N, k, im2), face_val(fs, v[k], N, k, im1), v0,
                          face_val(fs, v[k], N, k, ip1), face_val(fs, v[k], N, k, ip2));
        }
    }
    const double dp = p[self] - p[shifted(g, c, k, -1)];
    return nu * lap - dp + (k == axis ? G : 0.0);
}

/* Discrete divergence of cell c: sum_k v_k(c + e_k) - v_k(c). */
static double divergence(const grid *g, const uint8_t *fs, const double *const v[3], const int64_t c[3])
{
    const int64_t N = g->n[0] * g->n[1] * g->n[2];
    const int64_t self = at(g, c[0], c[1], c[2]);
    double d = 0.0;
    for (int k = 0; k < 3; ++k)
        d += face_val(fs, v[k], N, k, shifted(g, c, k, +1)) - face_val(fs, v[k], N, k, self);
    return d;
}

/*
 * One sweep: (u,v,w,p) -> (u2,v2,w2,p2).
 *   every fluid k-face:  v_k' = v_k + dt F_k(v, p);   solid faces: v_k' = 0
 *   every cell:          p'   = p - c2 dt div(v')
 */
void orc_sweep(const orc_params *prm, const uint8_t *fs, int64_t nx, int64_t ny, int64_t nz, int axis,
               const double *u, const double *v, const double *w, const double *p,
               double *u2, double *v2, double *w2, double *p2)
{
    grid g = {{nx, ny, nz}};
    const int64_t N = nx * ny * nz;
    const double nu = 1.0 / prm->re, dt = prm->dt, c2 = prm->c2, G = prm->drive;
    const double *vin[3] = {u, v, w};
    double *vout[3] = {u2, v2, w2};
    #pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t c[3] = {x, y, z};
                int64_t id = (z * ny + y) * nx + x;
                for (int k = 0; k < 3; ++k) {
                    if (fs[k * N + id]) {
                        vout[k][id] = 0.0;
                    } else {
                        double F = momentum(&g, fs, vin, p, k, c, axis, nu, G);
                        vout[k][id] = vin[k][id] + dt * F;
                    }
                }
            }
    const double *vnew[3] = {u2, v2, w2};
    #pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t c[3] = {x, y, z};
                int64_t id = (z * ny + y) * nx + x;
                if (prm->fixed_pressure && c[axis] == 0)
                    p2[id] = p[id];  /* fixed-pressure layer */
                else
                    p2[id] = p[id] - c2 * dt * divergence(&g, fs, vnew, c);
            }
}

/*
 * One sweep evaluated only at the listed cells (linear cell indices): writes
 * the four new values (u', v', w', p') of each listed cell to out[4*m + 0..3].
 * Used to check very large grids at sampled points.
 */
void orc_sweep_points(const orc_params *prm, const uint8_t *fs, int64_t nx, int64_t ny, int64_t nz,
                      int axis, const double *u, const double *v, const double *w, const double *p,
                      const int64_t *cells, int64_t ncells, double *out)
{
    grid g = {{nx, ny, nz}};
    const int64_t N = nx * ny * nz;
    const double nu = 1.0 / prm->re, dt = prm->dt, c2 = prm->c2, G = prm->drive;
    const double *vin[3] = {u, v, w};
    for (int64_t m = 0; m < ncells; ++m) {
        const int64_t id = cells[m];
        const int64_t c[3] = {id % nx, (id / nx) % ny, id / (nx * ny)};
        double vn[3];
        double div = 0.0;
        for (int k = 0; k < 3; ++k) {
            /* new value at the k-face of c and at the k-face of c + e_k */
            double lo, hi;
            if (fs[k * N + id]) lo = 0.0;
            else lo = vin[k][id] + dt * momentum(&g, fs, vin, p, k, c, axis, nu, G);
            int64_t up[3] = {c[0], c[1], c[2]};
            up[k] += 1;
            int64_t uid = at(&g, up[0], up[1], up[2]);
            int64_t upw[3] = {wrap(up[0], nx), wrap(up[1], ny), wrap(up[2], nz)};
            if (fs[k * N + uid]) hi = 0.0;
            else hi = vin[k][uid] + dt * momentum(&g, fs, vin, p, k, upw, axis, nu, G);
            vn[k] = lo;
            div += hi - lo;
        }
        out[4 * m + 0] = vn[0];
        out[4 * m + 1] = vn[1];
        out[4 * m + 2] = vn[2];
        out[4 * m + 3] = (prm->fixed_pressure && c[axis] == 0) ? p[id] : p[id] - c2 * dt * div;
    }
}

/*
 * Residual sums and fluxes of a state (v, p):
 *   out[0] = S_F = sum over fluid faces of F_k(v, p)^2
 *   out[1] = S_D = sum over cells of (nu div v)^2 (not over a fixed-pressure layer)
 *   out[2+k] = Q_k = sum over all k-faces of v_k (solid faces are zero)
 */
void orc_state_sums(const orc_params *prm, const uint8_t *fs, int64_t nx, int64_t ny, int64_t nz,
                    int axis, const double *u, const double *v, const double *w, const double *p,
                    double *out)
{
    grid g = {{nx, ny, nz}};
    const int64_t N = nx * ny * nz;
    const double nu = 1.0 / prm->re, G = prm->drive;
    const double *vin[3] = {u, v, w};
    double SF = 0.0, SD = 0.0, Q[3] = {0.0, 0.0, 0.0};
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t c[3] = {x, y, z};
                int64_t id = (z * ny + y) * nx + x;
                for (int k = 0; k < 3; ++k) {
                    if (fs[k * N + id]) continue;
                    double F = momentum(&g, fs, vin, p, k, c, axis, nu, G);
                    SF += F * F;
                    Q[k] += vin[k][id];
                }
                if (prm->fixed_pressure && c[axis] == 0) continue;  /* no mass balance there */
                double d = nu * divergence(&g, fs, vin, c);
                SD += d * d;
            }
    out[0] = SF;
    out[1] = SD;
    out[2] = Q[0];
    out[3] = Q[1];
    out[4] = Q[2];
}

/* Per-slice fluxes: qs[k][s] = sum of v_k over the k-faces with coordinate s
 * along axis k (qs is [3][max(nx,ny,nz)]). */
void orc_slice_flux(const uint8_t *fs, int64_t nx, int64_t ny, int64_t nz, const double *u,
                    const double *v, const double *w, double *qs)
{
    const int64_t N = nx * ny * nz;
    const int64_t L = nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz);
    const double *vin[3] = {u, v, w};
    for (int64_t i = 0; i < 3 * L; ++i) qs[i] = 0.0;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t id = (z * ny + y) * nx + x;
                int64_t s[3] = {x, y, z};
                for (int k = 0; k < 3; ++k)
                    if (!fs[k * N + id]) qs[k * L + s[k]] += vin[k][id];
            }
}

/* ------------------------------------------------------------------- solve */

/*
 * Solve for load axis `axis` (0 = x, 1 = y, 2 = z).
 *   fields u, v, w, p: [nz][ny][nx] FP64; on return they hold the state after
 *   `*sweeps` sweeps; with warm_start = 0 they are zeroed first.
 *   history (may be NULL): hist_sweep[cap], hist_r[cap], hist_eps[cap], hist_q[3*cap];
 *   *hist_n receives the number of records written.
 * Residual checks happen at sweep counts that are multiples of check_every
 * and at max_sweeps.  r = sqrt(S_F + S_D) / (G sqrt(N_f)), N_f = number of
 * fluid faces normal to the load axis (r = 1 for the state at rest).
 * Returns ORC_OK (r < tol, or eps_q < tol with stop_rule 1), ORC_NOT_CONVERGED,
 * ORC_DIVERGED (non-finite r or r > 1e3 min r), ORC_NO_FLOW, ORC_ERR_ARG, ORC_ERR_OOM.
 */
int orc_solve(const orc_params *prm, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz, int axis,
              double *u, double *v, double *w, double *p, int64_t cap, int64_t *hist_sweep,
              double *hist_r, double *hist_eps, double *hist_q, int64_t *hist_n, double *kcol,
              int64_t *sweeps)
{
    if (!prm || !mask || !u || !v || !w || !p || !kcol || !sweeps) return ORC_ERR_ARG;
    if (nx < 1 || ny < 1 || nz < 1 || axis < 0 || axis > 2) return ORC_ERR_ARG;
    if (!(prm->re > 0) || !(prm->c2 > 0) || !(prm->dt > 0) || !(prm->tol > 0) || !(prm->drive > 0) ||
        !(prm->voxel_size > 0) || prm->check_every < 1 || prm->max_sweeps < 0)
        return ORC_ERR_ARG;
    const int64_t N = nx * ny * nz;
    if (hist_n) *hist_n = 0;
    *sweeps = 0;

    uint8_t *fs = (uint8_t *)malloc(3 * (size_t)N);
    double *buf = (double *)malloc(4 * sizeof(double) * (size_t)N);
    if (!fs || !buf) { free(fs); free(buf); return ORC_ERR_OOM; }
    orc_face_solid(mask, nx, ny, nz, fs);

    int64_t nsolid = 0, nflow = 0;
    for (int64_t i = 0; i < N; ++i) {
        nsolid += mask[i] != 0;
        nflow += fs[axis * N + i] == 0;
    }
    if (nsolid == 0 || nflow == 0) { free(fs); free(buf); return ORC_NO_FLOW; }

    if (!prm->warm_start) {
        memset(u, 0, sizeof(double) * (size_t)N);
        memset(v, 0, sizeof(double) * (size_t)N);
        memset(w, 0, sizeof(double) * (size_t)N);
        memset(p, 0, sizeof(double) * (size_t)N);
    } else {
        double *f[3] = {u, v, w};
        for (int k = 0; k < 3; ++k)
            for (int64_t i = 0; i < N; ++i)
                if (fs[k * N + i]) f[k][i] = 0.0;
    }

    double *cur[4] = {u, v, w, p};
    double *nxt[4] = {buf, buf + N, buf + 2 * N, buf + 3 * N};
    const double G = prm->drive;
    const double scale = prm->voxel_size * prm->voxel_size / (prm->re * G * (double)N);
    double rmin = INFINITY, qprev = -1.0;
    int status = ORC_NOT_CONVERGED;
    int64_t n = 0;
    for (;;) {
        if (n % prm->check_every == 0 || n == prm->max_sweeps) {
            double s[5];
            orc_state_sums(prm, fs, nx, ny, nz, axis, cur[0], cur[1], cur[2], cur[3], s);
            double r = sqrt(s[0] + s[1]) / (G * sqrt((double)nflow));
            double qn = sqrt(s[2] * s[2] + s[3] * s[3] + s[4] * s[4]) / (double)N;
            double eps = (qprev >= 0.0 && qn > 0.0) ? fabs(qn - qprev) / qn : INFINITY;
            qprev = qn;
            if (hist_n && *hist_n < cap) {
                int64_t h = (*hist_n)++;
                if (hist_sweep) hist_sweep[h] = n;
                if (hist_r) hist_r[h] = r;
                if (hist_eps) hist_eps[h] = eps;
                if (hist_q)
                    for (int k = 0; k < 3; ++k) hist_q[3 * h + k] = s[2 + k] / (double)N;
            }
            for (int k = 0; k < 3; ++k) kcol[k] = s[2 + k] * scale;
            if (!isfinite(r) || r > 1e3 * rmin) { status = ORC_DIVERGED; break; }
            if (r < rmin) rmin = r;
            if ((prm->stop_rule == 0 && r < prm->tol) || (prm->stop_rule == 1 && eps < prm->tol)) {
                status = ORC_OK;
                break;
            }
            if (n >= prm->max_sweeps) { status = ORC_NOT_CONVERGED; break; }
        }
        orc_sweep(prm, fs, nx, ny, nz, axis, cur[0], cur[1], cur[2], cur[3], nxt[0], nxt[1], nxt[2],
                  nxt[3]);
        for (int f = 0; f < 4; ++f) { double *t = cur[f]; cur[f] = nxt[f]; nxt[f] = t; }
        ++n;
    }
    if (cur[0] != u) { /* the final state sits in the scratch buffer: copy back */
        memcpy(u, cur[0], sizeof(double) * (size_t)N);
        memcpy(v, cur[1], sizeof(double) * (size_t)N);
        memcpy(w, cur[2], sizeof(double) * (size_t)N);
        memcpy(p, cur[3], sizeof(double) * (size_t)N);
    }
    *sweeps = n;
    free(fs);
    free(buf);
    return status;
}

/* Timing helper for the CPU baseline: `count` sweeps from the state at rest;
 * returns the state after them in (u, v, w, p). */
int orc_run_sweeps(const orc_params *prm, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
                   int axis, int64_t count, double *u, double *v, double *w, double *p)
{
    const int64_t N = nx * ny * nz;
    uint8_t *fs = (uint8_t *)malloc(3 * (size_t)N);
    double *buf = (double *)malloc(4 * sizeof(double) * (size_t)N);
    if (!fs || !buf) { free(fs); free(buf); return ORC_ERR_OOM; }
    orc_face_solid(mask, nx, ny, nz, fs);
    double *cur[4] = {u, v, w, p};
    double *nxt[4] = {buf, buf + N, buf + 2 * N, buf + 3 * N};
    if (!prm->warm_start)
        for (int f = 0; f < 4; ++f) memset(cur[f], 0, sizeof(double) * (size_t)N);
    for (int64_t n = 0; n < count; ++n) {
        orc_sweep(prm, fs, nx, ny, nz, axis, cur[0], cur[1], cur[2], cur[3], nxt[0], nxt[1], nxt[2],
                  nxt[3]);
        for (int f = 0; f < 4; ++f) { double *t = cur[f]; cur[f] = nxt[f]; nxt[f] = t; }
    }
    if (cur[0] != u)
        for (int f = 0; f < 4; ++f) memcpy(f == 0 ? u : f == 1 ? v : f == 2 ? w : p, cur[f],
                                           sizeof(double) * (size_t)N);
    free(fs);
    free(buf);
    return ORC_OK;
}

/* Threads of the OpenMP loops (the CPU baseline times one thread and all). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
