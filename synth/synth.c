/*
 * Seeded synthetic porous-media masks.
 *
 * These generators stand in for the image data the method is applied to
 * (binarised XRCT volumes and microfluidic images): overlapping-sphere packings,
 * extruded 2-D ellipse packings with stochastic clogging, and Voronoi-strut
 * foams under uniaxial compression.  They contain none of the flow method's
 * arithmetic; the solver and its oracle both consume their output.
 *
 * Conventions shared by every generator:
 *   - mask layout uint8 [nz][ny][nx], x fastest; 1 = solid, 0 = pore;
 *   - a voxel (i,j,k) is represented by its centre (i+1/2, j+1/2, k+1/2);
 *   - distances use the periodic minimum image, so every mask is a true unit cell;
 *   - random numbers come from SplitMix64 (Steele, Lea, Flood, OOPSLA 2014),
 *     uniform doubles are (x >> 11) * 2^-53.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- RNG */

static uint64_t sm64_next(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static double sm64_uniform(uint64_t *s) { return (double)(sm64_next(s) >> 11) * 0x1.0p-53; }

/* Stateless draw for order-independent per-element randomness: one SplitMix64
 * output of a state built from (seed, stream, index). */
static uint64_t sm64_hash3(uint64_t seed, uint64_t stream, uint64_t index)
{
    uint64_t s = seed;
    uint64_t a = sm64_next(&s);          /* decorrelate the seed */
    s = a ^ (stream * 0xD6E8FEB86659FD93ULL);
    uint64_t b = sm64_next(&s);
    s = b ^ index;
    return sm64_next(&s);
}

uint64_t synth_splitmix64(uint64_t state_in, uint64_t *state_out)
{
    uint64_t s = state_in;
    uint64_t r = sm64_next(&s);
    if (state_out) *state_out = s;
    return r;
}

/* Minimum-image displacement along a periodic axis of length n, for
 * |d| < 3n/2 (every caller passes a difference of two coordinates in [0, n)). */
static double min_image(double d, double n)
{
    if (d > 0.5 * n) d -= n;
    else if (d < -0.5 * n) d += n;
    return d;
}

static int64_t wrapi(int64_t i, int64_t n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

/* ------------------------------------------------ overlapping spheres */

/*
 * Overlapping spheres with uniform centres in [0,nx)x[0,ny)x[0,nz) and radius
 * uniform in [rmin, rmax] (rmin == rmax gives a fixed radius).  Spheres are
 * added one at a time; generation stops at the first sphere after which the
 * porosity (pore fraction) is <= phi_target.  A voxel is solid when its centre
 * lies within distance r (inclusive) of a sphere centre, minimum image.
 *
 * The sequential definition is evaluated exactly but in parallel: a batch of
 * candidate spheres is drawn, every voxel records the smallest index of a
 * candidate covering it, and the stopping index follows from a histogram.
 * Returns the number of spheres used, or -1 on allocation failure / -2 when
 * the target cannot be reached within 2^26 spheres.
 */
int64_t synth_spheres(uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
                      double rmin, double rmax, double phi_target, uint64_t seed)
{
    const int64_t N = nx * ny * nz;
    const double rmean3 = (rmin == rmax) ? rmin * rmin * rmin
                          : (pow(rmax, 4) - pow(rmin, 4)) / (4.0 * (rmax - rmin));
    const double vmean = 4.0 / 3.0 * M_PI * rmean3;
    double lam = -log(phi_target > 1e-6 ? phi_target : 1e-6) / vmean * (double)N;
    int64_t ncand = (int64_t)(1.3 * lam) + 64;

    for (;;) {
        if (ncand > ((int64_t)1 << 26)) return -2;
        double *sc = (double *)malloc(sizeof(double) * 4 * (size_t)ncand);
        int32_t *minidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
        if (!sc || !minidx) { free(sc); free(minidx); return -1; }
        uint64_t st = seed;
        for (int64_t s = 0; s < ncand; ++s) {
            sc[4 * s + 0] = sm64_uniform(&st) * (double)nx;
            sc[4 * s + 1] = sm64_uniform(&st) * (double)ny;
            sc[4 * s + 2] = sm64_uniform(&st) * (double)nz;
            sc[4 * s + 3] = rmin + (rmax - rmin) * sm64_uniform(&st);
        }
        for (int64_t i = 0; i < N; ++i) minidx[i] = INT32_MAX;

        /* Each thread owns a contiguous range of z planes, so the min-stamping
         * below has a single writer per voxel. */
        #pragma omp parallel
        {
            int nth = 1, tid = 0;
#ifdef _OPENMP
            nth = omp_get_num_threads();
            tid = omp_get_thread_num();
#endif
            int64_t z0 = nz * tid / nth, z1 = nz * (tid + 1) / nth;
            for (int64_t s = 0; s < ncand && z0 < z1; ++s) {
                const double cx = sc[4 * s], cy = sc[4 * s + 1], cz = sc[4 * s + 2], r = sc[4 * s + 3];
                const double r2 = r * r;
                int64_t klo = (int64_t)floor(cz - r - 0.5) - 1, khi = (int64_t)ceil(cz + r - 0.5) + 1;
                int64_t jlo = (int64_t)floor(cy - r - 0.5) - 1, jhi = (int64_t)ceil(cy + r - 0.5) + 1;
                int64_t ilo = (int64_t)floor(cx - r - 0.5) - 1, ihi = (int64_t)ceil(cx + r - 0.5) + 1;
                if (khi - klo + 1 > nz) { klo = 0; khi = nz - 1; }
                if (jhi - jlo + 1 > ny) { jlo = 0; jhi = ny - 1; }
                if (ihi - ilo + 1 > nx) { ilo = 0; ihi = nx - 1; }
                for (int64_t kk = klo; kk <= khi; ++kk) {
                    int64_t k = wrapi(kk, nz);
                    if (k < z0 || k >= z1) continue;
                    double dz = min_image((double)k + 0.5 - cz, (double)nz);
                    double dz2 = dz * dz;
                    if (dz2 > r2) continue;
                    for (int64_t jj = jlo; jj <= jhi; ++jj) {
                        int64_t j = wrapi(jj, ny);
                        double dy = min_image((double)j + 0.5 - cy, (double)ny);
                        double dyz2 = dy * dy + dz2;
                        if (dyz2 > r2) continue;
                        int32_t *row = minidx + (k * ny + j) * nx;
                        for (int64_t ii = ilo; ii <= ihi; ++ii) {
                            int64_t i = wrapi(ii, nx);
                            double dx = min_image((double)i + 0.5 - cx, (double)nx);
                            if (dx * dx + dyz2 <= r2 && row[i] > (int32_t)s) row[i] = (int32_t)s;
                        }
                    }
                }
            }
        }

        /* covered(n) = #voxels whose smallest covering index is < n */
        int64_t *hist = (int64_t *)calloc((size_t)ncand + 1, sizeof(int64_t));
        if (!hist) { free(sc); free(minidx); return -1; }
        for (int64_t i = 0; i < N; ++i) {
            int32_t m = minidx[i];
            hist[m == INT32_MAX ? ncand : m] += 1;
        }
        int64_t covered = 0, nstop = -1;
        for (int64_t n = 1; n <= ncand; ++n) {
            covered += hist[n - 1];
            /* porosity <= target  <=>  (N - covered) <= phi_target * N */
            if ((double)(N - covered) <= phi_target * (double)N) { nstop = n; break; }
        }
        free(hist);
        if (nstop < 0) {            /* not enough candidates: draw more */
            free(sc); free(minidx);
            ncand *= 2;
            continue;
        }
        for (int64_t i = 0; i < N; ++i) mask[i] = (minidx[i] < nstop) ? 1 : 0;
        free(sc); free(minidx);
        return nstop;
    }
}

/* ------------------------------------------ 2-D ellipses + clogging */

/*
 * 2-D overlapping ellipses on an nx x ny periodic image: uniform centres,
 * semi-axes a, b uniform in [amin, amax], orientation uniform in [0, pi).
 * Pixel solid iff its centre satisfies (x'/a)^2 + (y'/b)^2 <= 1 in the
 * ellipse frame (minimum image).  Added one at a time until porosity <= target.
 * Writes img[ny][nx]; returns #ellipses used (or <0 on failure).
 */
int64_t synth_ellipses2d(uint8_t *img, int64_t nx, int64_t ny, double amin, double amax,
                         double phi_target, uint64_t seed)
{
    const int64_t N = nx * ny;
    memset(img, 0, (size_t)N);
    int64_t solid = 0;
    uint64_t st = seed;
    int64_t n = 0;
    while ((double)(N - solid) > phi_target * (double)N) {
        if (n > 10000000) return -2;
        double cx = sm64_uniform(&st) * (double)nx;
        double cy = sm64_uniform(&st) * (double)ny;
        double a = amin + (amax - amin) * sm64_uniform(&st);
        double b = amin + (amax - amin) * sm64_uniform(&st);
        double th = M_PI * sm64_uniform(&st);
        double c = cos(th), s = sin(th);
        double R = (a > b ? a : b) + 1.0;
        int64_t jlo = (int64_t)floor(cy - R), jhi = (int64_t)ceil(cy + R);
        int64_t ilo = (int64_t)floor(cx - R), ihi = (int64_t)ceil(cx + R);
        if (jhi - jlo + 1 > ny) { jlo = 0; jhi = ny - 1; }
        if (ihi - ilo + 1 > nx) { ilo = 0; ihi = nx - 1; }
        for (int64_t jj = jlo; jj <= jhi; ++jj) {
            int64_t j = wrapi(jj, ny);
            double dy = min_image((double)j + 0.5 - cy, (double)ny);
            for (int64_t ii = ilo; ii <= ihi; ++ii) {
                int64_t i = wrapi(ii, nx);
                double dx = min_image((double)i + 0.5 - cx, (double)nx);
                double xp = c * dx + s * dy, yp = -s * dx + c * dy;
                if ((xp / a) * (xp / a) + (yp / b) * (yp / b) <= 1.0 && !img[j * nx + i]) {
                    img[j * nx + i] = 1;
                    ++solid;
                }
            }
        }
        ++n;
    }
    return n;
}

/*
 * Stochastic clogging: `passes` synchronous dilation passes on a periodic 2-D
 * image.  In pass q every pore pixel with at least one solid 4-neighbour
 * (as of the start of the pass) turns solid with probability 1/2, drawn from
 * sm64_hash3(seed, q, pixel index).  Operates in place.
 */
void synth_clog2d(uint8_t *img, int64_t nx, int64_t ny, int passes, uint64_t seed)
{
    const int64_t N = nx * ny;
    uint8_t *prev = (uint8_t *)malloc((size_t)N);
    if (!prev) return;
    for (int q = 0; q < passes; ++q) {
        memcpy(prev, img, (size_t)N);
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t id = j * nx + i;
                if (prev[id]) continue;
                int nb = prev[j * nx + wrapi(i - 1, nx)] | prev[j * nx + wrapi(i + 1, nx)] |
                         prev[wrapi(j - 1, ny) * nx + i] | prev[wrapi(j + 1, ny) * nx + i];
                if (nb && (sm64_hash3(seed, (uint64_t)q, (uint64_t)id) >> 63)) img[id] = 1;
            }
    }
    free(prev);
}

/* Extrude a 2-D image to nz = depth + 2 planes: z = 0 and z = depth+1 are solid
 * walls, planes 1..depth copy the image.  out is [depth+2][ny][nx]. */
void synth_extrude(const uint8_t *img, int64_t nx, int64_t ny, int64_t depth, uint8_t *out)
{
    const int64_t P = nx * ny;
    memset(out, 1, (size_t)P);
    for (int64_t z = 1; z <= depth; ++z) memcpy(out + z * P, img, (size_t)P);
    memset(out + (depth + 1) * P, 1, (size_t)P);
}

/* -------------------------------------------------- Voronoi-strut foam */

/*
 * Open-cell foam: nseeds uniform seeds in the periodic box.  A voxel is solid
 * when its distance to the Voronoi edge of its three nearest seeds (s1,s2,s3,
 * minimum image) is <= radius.  That edge lies on the line where the bisector
 * planes of (s1,s2) and (s1,s3) intersect; the distance is measured to that
 * line.  Writes mask[nz][ny][nx].
 */
void synth_foam(uint8_t *mask, int64_t nx, int64_t ny, int64_t nz, int nseeds,
                double radius, uint64_t seed)
{
    double *sd = (double *)malloc(sizeof(double) * 3 * (size_t)nseeds);
    if (!sd) return;
    uint64_t st = seed;
    for (int s = 0; s < nseeds; ++s) {
        sd[3 * s + 0] = sm64_uniform(&st) * (double)nx;
        sd[3 * s + 1] = sm64_uniform(&st) * (double)ny;
        sd[3 * s + 2] = sm64_uniform(&st) * (double)nz;
    }
    const double r2 = radius * radius;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nz; ++k) {
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                double p[3] = {(double)i + 0.5, (double)j + 0.5, (double)k + 0.5};
                /* three nearest seeds, displacement vectors seed - p (minimum image) */
                double best[3] = {1e300, 1e300, 1e300};
                double vec[3][3] = {{0}};
                for (int s = 0; s < nseeds; ++s) {
                    double d0 = min_image(sd[3 * s] - p[0], (double)nx);
                    double d1 = min_image(sd[3 * s + 1] - p[1], (double)ny);
                    double d2 = min_image(sd[3 * s + 2] - p[2], (double)nz);
                    double dd = d0 * d0 + d1 * d1 + d2 * d2;
                    if (dd < best[2]) {
                        int at = (dd < best[0]) ? 0 : (dd < best[1]) ? 1 : 2;
                        for (int m = 2; m > at; --m) {
                            best[m] = best[m - 1];
                            vec[m][0] = vec[m - 1][0]; vec[m][1] = vec[m - 1][1]; vec[m][2] = vec[m - 1][2];
                        }
                        best[at] = dd;
                        vec[at][0] = d0; vec[at][1] = d1; vec[at][2] = d2;
                    }
                }
                /* Work in coordinates with p at the origin; seed a = vec[0], b, c.
                 * Bisector plane (a,b): n1 . x = h1 with n1 = b - a, h1 = (|b|^2 - |a|^2)/2. */
                double n1[3], n2[3];
                for (int m = 0; m < 3; ++m) { n1[m] = vec[1][m] - vec[0][m]; n2[m] = vec[2][m] - vec[0][m]; }
                double h1 = 0.5 * (best[1] - best[0]), h2 = 0.5 * (best[2] - best[0]);
                double dir[3] = {n1[1] * n2[2] - n1[2] * n2[1], n1[2] * n2[0] - n1[0] * n2[2],
                                 n1[0] * n2[1] - n1[1] * n2[0]};
                double dd = dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2];
                uint8_t solid = 0;
                if (dd > 1e-18) {
                    /* Closest point of the line to the origin: x0 = (h1 (n2 x d) + h2 (d x n1)) / |d|^2 */
                    double n2xd[3] = {n2[1] * dir[2] - n2[2] * dir[1], n2[2] * dir[0] - n2[0] * dir[2],
                                      n2[0] * dir[1] - n2[1] * dir[0]};
                    double dxn1[3] = {dir[1] * n1[2] - dir[2] * n1[1], dir[2] * n1[0] - dir[0] * n1[2],
                                      dir[0] * n1[1] - dir[1] * n1[0]};
                    double x0[3];
                    for (int m = 0; m < 3; ++m) x0[m] = (h1 * n2xd[m] + h2 * dxn1[m]) / dd;
                    double dist2 = x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2];
                    solid = dist2 <= r2;
                }
                mask[(k * ny + j) * nx + i] = solid;
            }
    }
    free(sd);
}

/* Nearest-neighbour rescale along z from nz_src to nz_dst planes:
 * z_src = floor((z + 1/2) * nz_src / nz_dst). */
void synth_rescale_z(const uint8_t *src, int64_t nx, int64_t ny, int64_t nz_src,
                     int64_t nz_dst, uint8_t *dst)
{
    const int64_t P = nx * ny;
    for (int64_t z = 0; z < nz_dst; ++z) {
        int64_t zs = (int64_t)floor(((double)z + 0.5) * (double)nz_src / (double)nz_dst);
        if (zs >= nz_src) zs = nz_src - 1;
        memcpy(dst + z * P, src + zs * P, (size_t)P);
    }
}

/* ---------------------------------------------------------------- rotated ellipsoid */

/*
 * One solid ellipsoid centred in an nx x ny x nz periodic box, semi-axes a, b,
 * c along e1, e2, e3 before it is turned about e1 by alpha (radians): the
 * benchmark geometry of the principal-direction study (100^3 box, a = c = 35,
 * b = 10).  A voxel is solid iff its centre p, relative to the box centre and
 * turned back by -alpha, satisfies (x/a)^2 + (y'/b)^2 + (z'/c)^2 <= 1 with
 * y' = cos(alpha) y + sin(alpha) z, z' = -sin(alpha) y + cos(alpha) z (minimum
 * image, so a body wider than the box wraps around).
 */
void synth_ellipsoid(uint8_t *mask, int64_t nx, int64_t ny, int64_t nz, double a, double b, double c,
                     double alpha)
{
    const double ca = cos(alpha), sa = sin(alpha);
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const double x = min_image((double)i + 0.5 - 0.5 * (double)nx, (double)nx);
                const double y = min_image((double)j + 0.5 - 0.5 * (double)ny, (double)ny);
                const double z = min_image((double)k + 0.5 - 0.5 * (double)nz, (double)nz);
                const double yr = ca * y + sa * z, zr = -sa * y + ca * z;
                const double q = (x / a) * (x / a) + (yr / b) * (yr / b) + (zr / c) * (zr / c);
                mask[(k * ny + j) * nx + i] = q <= 1.0;
            }
}
