// porestokes device kernels for gfx950 (MI355X).
//
//   face_bits / face_codes  mask -> face flags and per-cell stencil codes
//                           ("Evaluate neighborhood", Algorithm 1; §4, App. B)
//   fused sweep             one HBM pass per pseudo-time step (§3, Algorithm 1)
//   simple sweep            two-pass reference of the same arithmetic
//   state sums              FP64 residual and flux sums (convergence, Darcy)
#include "common.h"
#include "kernels.h"

#define GLOBAL_AS __attribute__((address_space(1)))

namespace ps {

// ============================================================== preprocessing

__device__ __forceinline__ int wrap_small(int i, int n)
{
    // i in (-3n, 3n): cheap periodic wrap for stencil offsets
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
}

__device__ __forceinline__ bool face_solid(const uint8_t *__restrict__ mask, int nx, int ny, int nz,
                                           int k, int x, int y, int z)
{
    x = wrap_small(x, nx);
    y = wrap_small(y, ny);
    z = wrap_small(z, nz);
    int bx = x, by = y, bz = z;
    if (k == 0) bx = wrap_small(x - 1, nx);
    else if (k == 1) by = wrap_small(y - 1, ny);
    else bz = wrap_small(z - 1, nz);
    const int64_t plane = (int64_t)nx * ny;
    return mask[z * plane + (int64_t)y * nx + x] != 0 || mask[bz * plane + (int64_t)by * nx + bx] != 0;
}

__global__ void k_face_bits(const uint8_t *__restrict__ mask, int nx, int ny, int nz, int W,
                            uint32_t *__restrict__ bits)
{
    const int64_t nwords = (int64_t)W * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * nwords) return;
    const int k = (int)(t / nwords);
    int64_t r = t % nwords;
    const int w = (int)(r % W);
    r /= W;
    const int y = (int)(r % ny);
    const int z = (int)(r / ny);
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
        const int x = w * 32 + b;
        if (x < nx && face_solid(mask, nx, ny, nz, k, x, y, z)) word |= 1u << b;
    }
    bits[t] = word;
}

// 3-bit stencil code from the solid flags at offsets -2, -1, +1, +2.
__device__ __forceinline__ uint32_t make_code(bool sm2, bool sm1, bool sp1, bool sp2)
{
    const bool far = (sm1 && !sp1) ? sp2 : ((sp1 && !sm1) ? sm2 : false);
    return (uint32_t)sm1 | ((uint32_t)sp1 << 1) | ((uint32_t)far << 2);
}

__global__ void k_face_codes(const uint8_t *__restrict__ mask, int nx, int ny, int nz,
                             uint32_t *__restrict__ codes)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int x = (int)(t % nx);
    const int y = (int)((t / nx) % ny);
    const int z = (int)(t / ((int64_t)nx * ny));
    uint32_t word = 0;
    for (int k = 0; k < 3; ++k) {
        // perpendicular axes in order: u -> (y, z), v -> (x, z), w -> (x, y)
        const int i1 = (k == 0) ? 1 : 0;
        const int i2 = (k == 2) ? 1 : 2;
        uint32_t c = 0;
        for (int pi = 0; pi < 2; ++pi) {
            const int i = pi == 0 ? i1 : i2;
            bool s[4];
            const int offs[4] = {-2, -1, 1, 2};
            for (int j = 0; j < 4; ++j) {
                int q[3] = {x, y, z};
                q[i] += offs[j];
                s[j] = face_solid(mask, nx, ny, nz, k, q[0], q[1], q[2]);
            }
            c |= make_code(s[0], s[1], s[2], s[3]) << (3 * pi);
        }
        if (face_solid(mask, nx, ny, nz, k, x, y, z)) c |= kSolidBit;
        word |= c << (kCodeBits * k);
    }
    codes[t] = word;
}

__global__ void k_counts(const uint8_t *__restrict__ mask, const uint32_t *__restrict__ codes, int64_t n,
                         unsigned long long *__restrict__ counts)
{
    __shared__ unsigned long long sc[4];
    if (threadIdx.x < 4) sc[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long c[4] = {0, 0, 0, 0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        c[0] += mask[t] != 0;
        const uint32_t w = codes[t];
        for (int k = 0; k < 3; ++k) c[1 + k] += ((w >> (kCodeBits * k)) & kSolidBit) == 0;
    }
    for (int i = 0; i < 4; ++i) atomicAdd(&sc[i], c[i]);
    __syncthreads();
    if (threadIdx.x < 4) atomicAdd(&counts[threadIdx.x], sc[threadIdx.x]);
}

template <typename T>
__global__ void k_zero_solid(const uint32_t *__restrict__ codes, int64_t n, T *__restrict__ u,
                             T *__restrict__ v, T *__restrict__ w)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t c = codes[t];
    if (c & kSolidBit) u[t] = T(0);
    if ((c >> kCodeBits) & kSolidBit) v[t] = T(0);
    if ((c >> (2 * kCodeBits)) & kSolidBit) w[t] = T(0);
}

template <typename S, typename D>
__global__ void k_convert(const S *__restrict__ src, D *__restrict__ dst, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dst[t] = (D)src[t];
}

// FP32 correction added into the FP64 state
__global__ void k_add_f32_to_f64(const float *__restrict__ src, double *__restrict__ dst, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dst[t] += (double)src[t];
}

// increment of one FP64 sweep, t - s0, rounded to FP32
__global__ void k_defect(const double *__restrict__ t_, const double *__restrict__ s0, float *__restrict__ d,
                         int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) d[t] = (float)(t_[t] - s0[t]);
}

static inline unsigned grid1d(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_face_bits(const uint8_t *mask, int nx, int ny, int nz, uint32_t *bits, hipStream_t s)
{
    const int W = (nx + 31) / 32;
    const int64_t total = 3LL * W * ny * nz;
    hipLaunchKernelGGL(k_face_bits, dim3(grid1d(total, 256)), dim3(256), 0, s, mask, nx, ny, nz, W, bits);
    return hipGetLastError();
}

hipError_t launch_face_codes(const uint8_t *mask, int nx, int ny, int nz, uint32_t *codes, hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL(k_face_codes, dim3(grid1d(n, 256)), dim3(256), 0, s, mask, nx, ny, nz, codes);
    return hipGetLastError();
}

hipError_t launch_counts(const uint8_t *mask, const uint32_t *codes, int64_t n, unsigned long long *counts,
                         hipStream_t s)
{
    hipError_t e = hipMemsetAsync(counts, 0, 4 * sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_counts, dim3((unsigned)blocks), dim3(256), 0, s, mask, codes, n, counts);
    return hipGetLastError();
}

hipError_t launch_zero_solid(Prec prec, const uint32_t *codes, int64_t n, void *u, void *v, void *w,
                             hipStream_t s)
{
    if (prec == kF64)
        hipLaunchKernelGGL(k_zero_solid<double>, dim3(grid1d(n, 256)), dim3(256), 0, s, codes, n,
                           (double *)u, (double *)v, (double *)w);
    else
        hipLaunchKernelGGL(k_zero_solid<float>, dim3(grid1d(n, 256)), dim3(256), 0, s, codes, n,
                           (float *)u, (float *)v, (float *)w);
    return hipGetLastError();
}

// ---- outer walls: the grid with solid layers appended along some axes

__global__ void k_pad_mask(const uint8_t *__restrict__ src, int nx, int ny, int nz, uint8_t *__restrict__ dst,
                           int px, int py, int pz)
{
    const int64_t n = (int64_t)px * py * pz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int x = (int)(t % px), y = (int)((t / px) % py), z = (int)(t / ((int64_t)px * py));
    dst[t] = (x < nx && y < ny && z < nz) ? src[((int64_t)z * ny + y) * nx + x] : (uint8_t)1;
}

// padded[t] = field at the same (x, y, z) inside the caller's grid, 0 in the added layers
template <typename T>
__global__ void k_embed(const T *__restrict__ src, int nx, int ny, int nz, T *__restrict__ dst, int px, int py,
                        int pz)
{
    const int64_t n = (int64_t)px * py * pz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int x = (int)(t % px), y = (int)((t / px) % py), z = (int)(t / ((int64_t)px * py));
    dst[t] = (x < nx && y < ny && z < nz) ? src[((int64_t)z * ny + y) * nx + x] : T(0);
}

template <typename T>
__global__ void k_extract(const T *__restrict__ src, int px, int py, T *__restrict__ dst, int nx, int ny, int nz)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int x = (int)(t % nx), y = (int)((t / nx) % ny), z = (int)(t / ((int64_t)nx * ny));
    dst[t] = src[((int64_t)z * py + y) * px + x];
}

hipError_t launch_pad_mask(const uint8_t *src, int nx, int ny, int nz, uint8_t *dst, int px, int py, int pz,
                           hipStream_t s)
{
    const int64_t n = (int64_t)px * py * pz;
    hipLaunchKernelGGL(k_pad_mask, dim3(grid1d(n, 256)), dim3(256), 0, s, src, nx, ny, nz, dst, px, py, pz);
    return hipGetLastError();
}

hipError_t launch_embed(size_t elem, const void *src, int nx, int ny, int nz, void *dst, int px, int py, int pz,
                        hipStream_t s)
{
    const int64_t n = (int64_t)px * py * pz;
    if (elem == sizeof(double))
        hipLaunchKernelGGL(k_embed<double>, dim3(grid1d(n, 256)), dim3(256), 0, s, (const double *)src, nx, ny, nz,
                           (double *)dst, px, py, pz);
    else
        hipLaunchKernelGGL(k_embed<float>, dim3(grid1d(n, 256)), dim3(256), 0, s, (const float *)src, nx, ny, nz,
                           (float *)dst, px, py, pz);
    return hipGetLastError();
}

hipError_t launch_extract(size_t elem, const void *src, int px, int py, void *dst, int nx, int ny, int nz,
                          hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny * nz;
    if (elem == sizeof(double))
        hipLaunchKernelGGL(k_extract<double>, dim3(grid1d(n, 256)), dim3(256), 0, s, (const double *)src, px, py,
                           (double *)dst, nx, ny, nz);
    else
        hipLaunchKernelGGL(k_extract<float>, dim3(grid1d(n, 256)), dim3(256), 0, s, (const float *)src, px, py,
                           (float *)dst, nx, ny, nz);
    return hipGetLastError();
}

// ---- mirroring: each selected axis doubled by the sample's mirror image

__global__ void k_mirror(const uint8_t *__restrict__ src, int nx, int ny, int nz, int axes, uint8_t *__restrict__ dst,
                         int mx, int my, int mz)
{
    const int64_t n = (int64_t)mx * my * mz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int x = (int)(t % mx), y = (int)((t / mx) % my), z = (int)(t / ((int64_t)mx * my));
    if ((axes & 1) && x >= nx) x = 2 * nx - 1 - x;
    if ((axes & 2) && y >= ny) y = 2 * ny - 1 - y;
    if ((axes & 4) && z >= nz) z = 2 * nz - 1 - z;
    dst[t] = src[((int64_t)z * ny + y) * nx + x];
}

hipError_t launch_mirror(const uint8_t *src, int nx, int ny, int nz, int axes, uint8_t *dst, hipStream_t s)
{
    const int mx = (axes & 1) ? 2 * nx : nx, my = (axes & 2) ? 2 * ny : ny, mz = (axes & 4) ? 2 * nz : nz;
    const int64_t n = (int64_t)mx * my * mz;
    hipLaunchKernelGGL(k_mirror, dim3(grid1d(n, 256)), dim3(256), 0, s, src, nx, ny, nz, axes, dst, mx, my, mz);
    return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double *src, float *dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL((k_convert<double, float>), dim3(grid1d(n, 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_f32_to_f64(const float *src, double *dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL((k_convert<float, double>), dim3(grid1d(n, 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_add_f32_to_f64(const float *src, double *dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_f32_to_f64, dim3(grid1d(n, 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_defect(const double *t, const double *s0, float *d, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_defect, dim3(grid1d(n, 256)), dim3(256), 0, s, t, s0, d, n);
    return hipGetLastError();
}

// ============================================================== fused sweep
//
// One launch advances every instance of the table by one sweep, fusing the
// pressure update of sweep n with the velocity update of sweep n+1:
//
//   in:  v^n (velocity set n&1), p^{n-1} (pressure set n&1)
//   p^n     = p^{n-1} - c2 dt div(v^n)                    (skip: p^n = p^{n-1})
//   v^{n+1} = v^n + dt F(v^n, p^n) on fluid faces, 0 on solid faces
//   out: p^n, v^{n+1} (the other sets)
//
// This reads and writes each of the four fields once per sweep (the
// velocity-then-pressure order of Algorithm 1 regrouped), and the residual of
// the state (v^n, p^n) -- F(v^n, p^n) and div v^n -- falls out of the same pass.
//
// Work decomposition: a workgroup owns a TX x TY column tile of the x-y plane
// and a chunk of zc planes, streamed bottom to top, one thread per column.
// Per plane, u, v and p^{n-1} are staged in LDS with a two-cell halo (the
// App. B stencils reach two faces across the flow); w is staged one plane
// ahead.  The planes above and below each thread's own column stay in a
// register window (5 planes of u and v, 3 of w).  Each thread computes p^n of
// its own cell and of its -x and -y neighbours (the pressure gradient of a
// face reads the cell behind it), so pressures are never exchanged.  LDS
// slots rotate (u, v, p over 2 planes, w over 3), which leaves one barrier
// per plane.  Every global load -- own column and halo -- is issued one
// iteration before the plane it feeds is staged, behind the barrier and the
// arithmetic of the current plane (with 4-7 waves per SIMD that covers the
// HBM latency; loading two iterations ahead measured no faster and held 25
// more registers).
// Results and stencil codes are touched once per launch: their stores and
// loads are non-temporal, leaving L2 to the planes that neighbouring tiles
// read again as halo.

// The far-wall coefficient of App. B (-1/5, on v[+2] when the near wall is
// at -1, on v[-2] when it is at +1) is nonzero for exactly two codes, so the
// LDS table holds (a, b) only -- one 16-byte read per lookup in FP64 instead
// of two -- and gp, gm come from two compares.  Same values, same operation
// order as d2_perp: the result is bitwise the same.
template <typename T>
struct CoefAB {
    T a, b;
};

template <typename T>
__device__ __forceinline__ T d2_perp_tab(const CoefAB<T> *tab, uint32_t c, T vm2, T vm1, T v0, T vp1, T vp2)
{
    const CoefAB<T> ab = tab[c];
    const T far = -(T(1) / T(5));
    const T gp = c == 1u ? far : T(0);
    const T gm = c == 2u ? far : T(0);
    T t = gm * vm2;
    t = fma(gp, vp2, t);
    t = fma(ab.b, v0, t);
    return fma(ab.a, vm1 + vp1, t);
}

template <bool B>
struct BoolC {
    static constexpr bool value = B;
};

// MI355X: 8 XCDs of 32 CUs; workgroup i of a dispatch goes to XCD i mod 8.
constexpr int kNumXcd = 8;
constexpr int kCusPerXcd = 32;

template <typename T, int TX, int TY>
struct FusedShared {
    static constexpr int PX = TX + 4, PY = TY + 4, PP = PX * PY;
    T u[2][PP];
    T v[2][PP];
    T p[2][PP];
    T w[3][PP];
    CoefAB<T> tab[8];
    double red[kNumSums * (TX * TY / 64)];
};

// RED: accumulate the residual and flux sums of the state (the launches at a
// convergence check); the other launches carry no accumulators, which keeps
// the FP64 64x16 variant within 128 VGPRs.
//
// SRC: the correction form.  The state is a correction e to a fixed state s0
// and the sweep is e <- A e + d0, where A is the sweep without the drive and
// d0 = T(s0) - s0 is the increment of the full sweep T at s0: the pressure
// gradient uses p^n without d0, and d0 is added to u, v, w and p^n as they
// are stored.  The fixed point is e* = s* - s0.  The residual of s0 + e
// follows from linearity: F(s0 + e) = F_A(e) + d0_v / dt and
// div(v0 + e_v) = div(e_v) - d0_p / (c2 dt); the flux sums are those of e.
template <typename T, int TX, int TY, bool RED, bool SRC = false>
__global__ void __launch_bounds__(TX *TY)
k_fused(const InstDev *__restrict__ insts, int ninst, int parity)
{
    constexpr int NT = TX * TY;
    constexpr int PX = TX + 4, PY = TY + 4;
    constexpr int NHALO = PX * PY - NT;
    static_assert(NHALO <= NT, "one halo position per thread");
    __shared__ FusedShared<T, TX, TY> sh;

    // ---- XCD-aware order: workgroups are dispatched round-robin over the
    // XCDs, each with its own L2.  Give each XCD a contiguous run of tiles so
    // that the halo reads of neighbouring tiles hit the L2 that loaded them.
    // With many tiles per plane the runs of all eight XCDs start at the same
    // in-plane tile of different z-chunks, and the XCDs then stream the same
    // in-plane region at once; starting XCD i's run 1/8 of its length later
    // for each i measured up to 12 % faster there (FP32, 1024^3) and 1-2 %
    // slower with 64 tiles per plane (256^3), hence the threshold.  Blocks are
    // only permuted: results are unchanged.
    //
    // FP64 workgroups of 1024 threads run one per CU (their LDS rings take
    // 98-114 KiB), so the chip holds 256 of them at a time.  For these the
    // order is round-major: workgroups 8 M r ... 8 M (r + 1) - 1 (M = 32 CUs
    // per XCD) form round r and take the contiguous tiles of that range, XCD i
    // the i-th run of 32.  Every round then has the layout of a launch of 256
    // tiles: 3-5 % faster than one run per XCD (three 256^3 instances, 1536^3).
    // Blocks are only permuted: results are unchanged.
    const int64_t nbk = gridDim.x, xcd = blockIdx.x % kNumXcd, kx = blockIdx.x / kNumXcd;
    int64_t b;
    if constexpr (sizeof(T) == 8 && TX * TY == 1024) {
        constexpr int64_t M = kCusPerXcd;
        const int64_t full = nbk / (kNumXcd * M);  // complete rounds
        if (kx / M < full) {
            b = (kx / M) * (kNumXcd * M) + xcd * M + (kx % M);
        } else {
            // the partial last round: one run per XCD over the remaining range
            const int64_t base = full * kNumXcd * M, nr = nbk - base;
            const int64_t qr = nr / kNumXcd, rr = nr % kNumXcd;
            b = base + (xcd < rr ? xcd * (qr + 1) : rr * (qr + 1) + (xcd - rr) * qr) + (kx - full * M);
        }
    } else {
        const int64_t q = nbk / kNumXcd, rem = nbk % kNumXcd;
        const int64_t qx = xcd < rem ? q + 1 : q;  // length of this XCD's run
        const bool rotate = (int64_t)insts[0].tiles_x * insts[0].tiles_y >= 256;
        b = (xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q) +
            (rotate ? (kx + xcd * (qx / kNumXcd)) % qx : kx);
    }

    // ---- instance of this block (ranges are sorted by blk_begin)
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (insts[mid].blk_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    const InstDev &I = insts[lo];
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const int64_t lb = b - I.blk_begin;
    const int bx = (int)(lb % I.tiles_x);
    const int64_t rr = lb / I.tiles_x;
    const int by = (int)(rr % I.tiles_y);
    const int bz = (int)(rr / I.tiles_y);
    const int x0 = bx * TX, y0 = by * TY;
    const int z0 = bz * I.zc;
    const int z1 = min(z0 + I.zc, nz);
    const int64_t plane = (int64_t)nx * ny;
    const int eff = parity ^ I.par_off;
    // Pointers read from the instance table are generic; placing them in the
    // global address space gives global (not flat) memory instructions, which
    // do not share a wait counter with LDS traffic.
    const T GLOBAL_AS *__restrict__ Uin = (const T GLOBAL_AS *)I.vel[eff][0];
    const T GLOBAL_AS *__restrict__ Vin = (const T GLOBAL_AS *)I.vel[eff][1];
    const T GLOBAL_AS *__restrict__ Win = (const T GLOBAL_AS *)I.vel[eff][2];
    const T GLOBAL_AS *__restrict__ Pin = (const T GLOBAL_AS *)I.pres[eff];
    T GLOBAL_AS *__restrict__ Uout = (T GLOBAL_AS *)I.vel[eff ^ 1][0];
    T GLOBAL_AS *__restrict__ Vout = (T GLOBAL_AS *)I.vel[eff ^ 1][1];
    T GLOBAL_AS *__restrict__ Wout = (T GLOBAL_AS *)I.vel[eff ^ 1][2];
    T GLOBAL_AS *__restrict__ Pout = (T GLOBAL_AS *)I.pres[eff ^ 1];
    const uint32_t GLOBAL_AS *__restrict__ codes = (const uint32_t GLOBAL_AS *)I.codes;
    const T GLOBAL_AS *__restrict__ Su = (const T GLOBAL_AS *)I.src[0];
    const T GLOBAL_AS *__restrict__ Sv = (const T GLOBAL_AS *)I.src[1];
    const T GLOBAL_AS *__restrict__ Sw = (const T GLOBAL_AS *)I.src[2];
    const T GLOBAL_AS *__restrict__ Sp = (const T GLOBAL_AS *)I.src[3];
    const T nu = (T)I.nu, dt = (T)I.dt, c2dt = (T)I.c2dt;
    const T gu = I.axis == 0 ? (T)I.drive : T(0);
    const T gv = I.axis == 1 ? (T)I.drive : T(0);
    const T gw = I.axis == 2 ? (T)I.drive : T(0);
    const bool skip = I.skip != 0;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    if (tid < 8) {
        const Coef<T> c8 = coef_of_code<T>(tid);
        sh.tab[tid] = {c8.a, c8.b};
    }

    // ---- own column (inactive threads hold the wrapped column: LDS stays periodic)
    const int gx = x0 + tx, gy = y0 + ty;
    const bool active = gx < nx && gy < ny;
    const int own = wrap_int(gy, ny) * nx + wrap_int(gx, nx);
    const int cl = (ty + 2) * PX + (tx + 2);  // own position in the padded plane

    // ---- halo position of this thread in the padded plane (ring of width 2)
    const bool has_halo = tid < NHALO;
    int hoff = 0, hlds = 0;
    bool has_ph = false;  // the -x column / -y row that p^{n-1} needs
    if (has_halo) {
        int px, py;
        if (tid < 2 * PX) {
            py = tid / PX;
            px = tid % PX;
        } else if (tid < 4 * PX) {
            const int hh = tid - 2 * PX;
            py = PY - 2 + hh / PX;
            px = hh % PX;
        } else {
            const int hh = tid - 4 * PX;
            py = 2 + hh / 4;
            const int c = hh % 4;
            px = c < 2 ? c : PX - 4 + c;
        }
        hlds = py * PX + px;
        hoff = wrap_int(y0 - 2 + py, ny) * nx + wrap_int(x0 - 2 + px, nx);
        has_ph = (px == 1 && py >= 2 && py <= TY + 1) || (py == 1 && px >= 2 && px <= TX + 1);
    }

    // ---- prime the registers for the prologue plane zz = z0 - 1
    T Uw[5], Vw[5], Ww[3];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const int64_t zo = (int64_t)wrap_int(z0 - 3 + j, nz) * plane + own;
        Uw[j] = Uin[zo];
        Vw[j] = Vin[zo];
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) Ww[j] = Win[(int64_t)wrap_int(z0 - 2 + j, nz) * plane + own];
    int zcur = wrap_int(z0 - 1, nz);  // zz
    int z1p = wrap_int(z0, nz);       // zz + 1
    int z2p = wrap_int(z0 + 1, nz);   // zz + 2
    int z3p = wrap_int(z0 + 2, nz);   // zz + 3
    T pold = Pin[(int64_t)zcur * plane + own];
    uint32_t code = 0;
    T sU = T(0), sV = T(0), sW = T(0), sP = T(0);  // correction-form terms of plane zz
    T hU = T(0), hV = T(0), hW = T(0), hP = T(0);
    if (has_halo) {
        hU = Uin[(int64_t)zcur * plane + hoff];
        hV = Vin[(int64_t)zcur * plane + hoff];
        hW = Win[(int64_t)z1p * plane + hoff];
        if (has_ph) hP = Pin[(int64_t)zcur * plane + hoff];
    }
    int slot = 0;                   // u, v, p slot of plane zz
    int wc = 0, wn = 1;             // w slots of planes zz and zz + 1
    T pn_prev = T(0);

    double acc[kNumSums] = {0.0, 0.0, 0.0, 0.0, 0.0};

    // One plane step; `body` is false for the prologue plane zz = z0 - 1, which
    // only primes p^n and the staged planes.  The prologue is peeled off so
    // that every step of the loop stores unconditionally: the vector-memory
    // counter (s_waitcnt vmcnt) counts loads and stores in issue order, and a
    // path without the stores made the compiler wait for each step's stores
    // to complete before the loads of the next plane could be used (10 %).
    auto plane_step = [&](const int zz, auto body_c) __attribute__((always_inline)) {
        constexpr bool body = decltype(body_c)::value;
        T *const su = sh.u[slot];
        T *const sv = sh.v[slot];
        T *const sp = sh.p[slot];
        T *const swc = sh.w[wc];
        T *const swn = sh.w[wn];

        // ---- stage plane zz (u, v, p) and plane zz + 1 (w)
        su[cl] = Uw[2];
        sv[cl] = Vw[2];
        sp[cl] = pold;
        swn[cl] = Ww[2];
        if (has_halo) {
            su[hlds] = hU;
            sv[hlds] = hV;
            swn[hlds] = hW;
            if (has_ph) sp[hlds] = hP;
        }

        // ---- loads for iteration zz + 1 (planes wrap, so every address is
        // valid); the last iteration of the chunk needs none
        const bool ahead = zz + 1 < z1;
        T bU = T(0), bV = T(0), bW = T(0), bP = T(0);
        T bSu = T(0), bSv = T(0), bSw = T(0), bSp = T(0);
        uint32_t bC = 0;
        if (ahead) {
            if constexpr (SRC) {
                const int64_t oa = (int64_t)z1p * plane + own;
                bSu = __builtin_nontemporal_load(&Su[oa]);
                bSv = __builtin_nontemporal_load(&Sv[oa]);
                bSw = __builtin_nontemporal_load(&Sw[oa]);
                bSp = __builtin_nontemporal_load(&Sp[oa]);
            }
            bU = Uin[(int64_t)z3p * plane + own];
            bV = Vin[(int64_t)z3p * plane + own];
            bW = Win[(int64_t)z2p * plane + own];
            bP = Pin[(int64_t)z1p * plane + own];
            bC = __builtin_nontemporal_load(&codes[(int64_t)z1p * plane + own]);
        }
        T bhU = T(0), bhV = T(0), bhW = T(0), bhP = T(0);
        if (has_halo && ahead) {
            bhU = Uin[(int64_t)z1p * plane + hoff];
            bhV = Vin[(int64_t)z1p * plane + hoff];
            bhW = Win[(int64_t)z2p * plane + hoff];
            if (has_ph) bhP = Pin[(int64_t)z1p * plane + hoff];
        }
        __syncthreads();

        // ---- p^n of the own cell
        const T dvg = divergence(Uw[2], su[cl + 1], Vw[2], sv[cl + PX], Ww[1], Ww[2]);
        const T pn = skip ? pold : fma(-c2dt, dvg, pold);

        if constexpr (body) {
            // lanes outside the grid hold a wrapped column: they compute and
            // store exactly the values of that column's own lane
            // p^n of the -x and -y neighbours, from the staged planes
            const T dxm = divergence(su[cl - 1], Uw[2], sv[cl - 1], sv[cl - 1 + PX], swc[cl - 1], swn[cl - 1]);
            const T pxm = skip ? sp[cl - 1] : fma(-c2dt, dxm, sp[cl - 1]);
            const T dym = divergence(su[cl - PX], su[cl - PX + 1], sv[cl - PX], Vw[2], swc[cl - PX], swn[cl - PX]);
            const T pym = skip ? sp[cl - PX] : fma(-c2dt, dym, sp[cl - PX]);
            const int64_t o = (int64_t)zcur * plane + own;
            __builtin_nontemporal_store(SRC ? pn + sP : pn, &Pout[o]);
            // u: own axis x, across y (LDS) and z (registers)
            const uint32_t cu = code;
            const T u0 = Uw[2];
            const T u_d2x = d2_own(su[cl - 1], u0, su[cl + 1]);
            const T u_d2y = d2_perp_tab(sh.tab, cu & 7, su[cl - 2 * PX], su[cl - PX], u0, su[cl + PX], su[cl + 2 * PX]);
            const T u_d2z = d2_perp_tab(sh.tab, (cu >> 3) & 7, Uw[0], Uw[1], u0, Uw[3], Uw[4]);
            const T Fu = momentum(u_d2x, u_d2y, u_d2z, pn, pxm, nu, gu);
            const bool su_ = (cu & kSolidBit) != 0;
            __builtin_nontemporal_store(su_ ? T(0) : (SRC ? fma(dt, Fu, u0) + sU : fma(dt, Fu, u0)),
                                        &Uout[o]);
            // v: own axis y, across x (LDS) and z (registers)
            const uint32_t cv = code >> kCodeBits;
            const T v0 = Vw[2];
            const T v_d2x = d2_perp_tab(sh.tab, cv & 7, sv[cl - 2], sv[cl - 1], v0, sv[cl + 1], sv[cl + 2]);
            const T v_d2y = d2_own(sv[cl - PX], v0, sv[cl + PX]);
            const T v_d2z = d2_perp_tab(sh.tab, (cv >> 3) & 7, Vw[0], Vw[1], v0, Vw[3], Vw[4]);
            const T Fv = momentum(v_d2x, v_d2y, v_d2z, pn, pym, nu, gv);
            const bool sv_ = (cv & kSolidBit) != 0;
            __builtin_nontemporal_store(sv_ ? T(0) : (SRC ? fma(dt, Fv, v0) + sV : fma(dt, Fv, v0)),
                                        &Vout[o]);
            // w: own axis z (registers), across x and y (LDS)
            const uint32_t cw = code >> (2 * kCodeBits);
            const T w0 = Ww[1];
            const T w_d2x = d2_perp_tab(sh.tab, cw & 7, swc[cl - 2], swc[cl - 1], w0, swc[cl + 1], swc[cl + 2]);
            const T w_d2y = d2_perp_tab(sh.tab, (cw >> 3) & 7, swc[cl - 2 * PX], swc[cl - PX], w0, swc[cl + PX],
                                    swc[cl + 2 * PX]);
            const T w_d2z = d2_own(Ww[0], w0, Ww[2]);
            const T Fw = momentum(w_d2x, w_d2y, w_d2z, pn, pn_prev, nu, gw);
            const bool sw_ = (cw & kSolidBit) != 0;
            __builtin_nontemporal_store(sw_ ? T(0) : (SRC ? fma(dt, Fw, w0) + sW : fma(dt, Fw, w0)),
                                        &Wout[o]);
            if (RED && !SRC && active) {
                const double fu = su_ ? 0.0 : (double)Fu, fv = sv_ ? 0.0 : (double)Fv,
                             fw = sw_ ? 0.0 : (double)Fw;
                acc[0] += fu * fu + fv * fv + fw * fw;
                const double nd = (double)(nu * dvg);
                acc[1] += nd * nd;
            }
            if (RED && SRC && active) {
                const double fu = su_ ? 0.0 : fma((double)sU, I.rdt, (double)Fu);
                const double fv = sv_ ? 0.0 : fma((double)sV, I.rdt, (double)Fv);
                const double fw = sw_ ? 0.0 : fma((double)sW, I.rdt, (double)Fw);
                acc[0] += fu * fu + fv * fv + fw * fw;
                const double nd = (double)nu * fma(-(double)sP, I.rc2dt, (double)dvg);
                acc[1] += nd * nd;
            }
            if (RED && active) {
                acc[2] += (double)u0;
                acc[3] += (double)v0;
                acc[4] += (double)w0;
            }
        }

        // ---- advance
        pn_prev = pn;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            Uw[j] = Uw[j + 1];
            Vw[j] = Vw[j + 1];
        }
        Uw[4] = bU;
        Vw[4] = bV;
        Ww[0] = Ww[1];
        Ww[1] = Ww[2];
        Ww[2] = bW;
        pold = bP;
        code = bC;
        sU = bSu;
        sV = bSv;
        sW = bSw;
        sP = bSp;
        hU = bhU;
        hV = bhV;
        hW = bhW;
        hP = bhP;
        zcur = z1p;
        z1p = z2p;
        z2p = z3p;
        z3p = (z3p + 1 == nz) ? 0 : z3p + 1;
        slot ^= 1;
        wc = wn;
        wn = (wn == 2) ? 0 : wn + 1;
    };
    plane_step(z0 - 1, BoolC<false>{});
    // the prologue's loads land in the registers the loop carries: complete
    // them here, or the loop head would wait as if they were still in flight
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0) expcnt(7) lgkmcnt(15)
    for (int zz = z0; zz < z1; ++zz) plane_step(zz, BoolC<true>{});
    if (RED) block_sums(acc, sh.red, I.partials + lb * kNumSums);
}

bool fused_alone(Prec prec, int tx, int ty, int64_t tiles_per_plane)
{
    return prec == kF32 && tx * ty == 1024 && tiles_per_plane >= 1024;
}

bool fused_tile_supported(int tx, int ty, int prec)
{
    // one halo position per thread; LDS rings within a workgroup's 160 KiB
    // (64x16 in FP64 takes 98 KiB: one workgroup of 16 waves per CU)
    (void)prec;
    return (tx == 128 && ty == 8) || (tx == 64 && (ty == 8 || ty == 16)) || (tx == 32 && (ty == 8 || ty == 16));
}

// Dynamic LDS (the kernel does not touch it) that takes a workgroup's share
// of the CU's 160 KiB past one half: one workgroup per CU.
template <typename T, int TX, int TY>
static unsigned one_per_cu_lds()
{
    constexpr size_t half = 80 * 1024, st = sizeof(FusedShared<T, TX, TY>);
    return st > half ? 0u : (unsigned)(half - st + 256);
}

template <typename T, bool SRC = false>
static hipError_t launch_fused_t(int tx, int ty, const InstDev *insts, int ninst, int64_t nblocks, int parity,
                                 int reduce, hipStream_t s, bool alone)
{
    const dim3 grid((unsigned)nblocks);
#define PS_FUSED_CASE(TX_, TY_)                                                                             \
    if (tx == TX_ && ty == TY_) {                                                                          \
        const unsigned dyn = alone ? one_per_cu_lds<T, TX_, TY_>() : 0u;                                   \
        if (reduce)                                                                                        \
            hipLaunchKernelGGL((k_fused<T, TX_, TY_, true, SRC>), grid, dim3(TX_ * TY_), dyn, s, insts,    \
                               ninst, parity);                                                             \
        else                                                                                               \
            hipLaunchKernelGGL((k_fused<T, TX_, TY_, false, SRC>), grid, dim3(TX_ * TY_), dyn, s, insts,   \
                               ninst, parity);                                                             \
        return hipGetLastError();                                                                          \
    }
    PS_FUSED_CASE(128, 8)
    PS_FUSED_CASE(64, 8)
    PS_FUSED_CASE(64, 16)
    PS_FUSED_CASE(32, 8)
    PS_FUSED_CASE(32, 16)
#undef PS_FUSED_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_fused(Prec prec, int tx, int ty, const InstDev *insts, int ninst, int64_t nblocks, int parity,
                        int reduce, hipStream_t s, bool alone)
{
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (!fused_tile_supported(tx, ty, prec)) return hipErrorInvalidValue;
    return prec == kF64 ? launch_fused_t<double>(tx, ty, insts, ninst, nblocks, parity, reduce, s, alone)
                        : launch_fused_t<float>(tx, ty, insts, ninst, nblocks, parity, reduce, s, alone);
}

hipError_t launch_fused_src(int tx, int ty, const InstDev *insts, int ninst, int64_t nblocks, int parity,
                            int reduce, hipStream_t s, bool alone)
{
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (!fused_tile_supported(tx, ty, kF32)) return hipErrorInvalidValue;
    return launch_fused_t<float, true>(tx, ty, insts, ninst, nblocks, parity, reduce, s, alone);
}

// ============================================================== reductions

__global__ void k_reduce_partials(const PartialRef *__restrict__ refs, double *__restrict__ out)
{
    __shared__ double scratch[kNumSums * 4];
    const PartialRef r = refs[blockIdx.x];
    double acc[kNumSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < r.nblocks; i += blockDim.x)
#pragma unroll
        for (int j = 0; j < kNumSums; ++j) acc[j] += r.partials[i * kNumSums + j];
    block_sums(acc, scratch, out + (int64_t)blockIdx.x * kNumSums);
}

hipError_t launch_reduce_partials(const PartialRef *refs, int ninst, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_partials, dim3(ninst), dim3(256), 0, s, refs, out);
    return hipGetLastError();
}

// ============================================================== simple sweep
//
// Velocity pass: one thread per cell updates its three faces from (v^n, p^n);
// pressure pass: p^{n+1} = p^n - c2 dt div(v^{n+1}).  Same per-face routines as
// the fused kernel; all neighbours come straight from global memory.

template <typename T>
__device__ __forceinline__ T ld(const T *__restrict__ f, int nx, int ny, int nz, int x, int y, int z)
{
    return f[((int64_t)wrap_small(z, nz) * ny + wrap_small(y, ny)) * nx + wrap_small(x, nx)];
}

template <typename T>
__global__ void k_simple_vel(int nx, int ny, int nz, int axis, const uint32_t *__restrict__ codes,
                             const T *__restrict__ U, const T *__restrict__ V, const T *__restrict__ W,
                             const T *__restrict__ P, T *__restrict__ Uo, T *__restrict__ Vo, T *__restrict__ Wo,
                             T nu, T dt, T drive)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int x = (int)(t % nx), y = (int)((t / nx) % ny), z = (int)(t / ((int64_t)nx * ny));
    const uint32_t code = codes[t];
    const T pc = P[t];
    {
        const uint32_t c = code;
        const T v0 = U[t];
        const T d2x = d2_own(ld(U, nx, ny, nz, x - 1, y, z), v0, ld(U, nx, ny, nz, x + 1, y, z));
        const T d2y = d2_perp(coef_of_code<T>(c & 7), ld(U, nx, ny, nz, x, y - 2, z), ld(U, nx, ny, nz, x, y - 1, z),
                              v0, ld(U, nx, ny, nz, x, y + 1, z), ld(U, nx, ny, nz, x, y + 2, z));
        const T d2z = d2_perp(coef_of_code<T>((c >> 3) & 7), ld(U, nx, ny, nz, x, y, z - 2),
                              ld(U, nx, ny, nz, x, y, z - 1), v0, ld(U, nx, ny, nz, x, y, z + 1),
                              ld(U, nx, ny, nz, x, y, z + 2));
        const T F = momentum(d2x, d2y, d2z, pc, ld(P, nx, ny, nz, x - 1, y, z), nu, axis == 0 ? drive : T(0));
        Uo[t] = (c & kSolidBit) ? T(0) : fma(dt, F, v0);
    }
    {
        const uint32_t c = code >> kCodeBits;
        const T v0 = V[t];
        const T d2x = d2_perp(coef_of_code<T>(c & 7), ld(V, nx, ny, nz, x - 2, y, z), ld(V, nx, ny, nz, x - 1, y, z),
                              v0, ld(V, nx, ny, nz, x + 1, y, z), ld(V, nx, ny, nz, x + 2, y, z));
        const T d2y = d2_own(ld(V, nx, ny, nz, x, y - 1, z), v0, ld(V, nx, ny, nz, x, y + 1, z));
        const T d2z = d2_perp(coef_of_code<T>((c >> 3) & 7), ld(V, nx, ny, nz, x, y, z - 2),
                              ld(V, nx, ny, nz, x, y, z - 1), v0, ld(V, nx, ny, nz, x, y, z + 1),
                              ld(V, nx, ny, nz, x, y, z + 2));
        const T F = momentum(d2x, d2y, d2z, pc, ld(P, nx, ny, nz, x, y - 1, z), nu, axis == 1 ? drive : T(0));
        Vo[t] = (c & kSolidBit) ? T(0) : fma(dt, F, v0);
    }
    {
        const uint32_t c = code >> (2 * kCodeBits);
        const T v0 = W[t];
        const T d2x = d2_perp(coef_of_code<T>(c & 7), ld(W, nx, ny, nz, x - 2, y, z), ld(W, nx, ny, nz, x - 1, y, z),
                              v0, ld(W, nx, ny, nz, x + 1, y, z), ld(W, nx, ny, nz, x + 2, y, z));
        const T d2y = d2_perp(coef_of_code<T>((c >> 3) & 7), ld(W, nx, ny, nz, x, y - 2, z),
                              ld(W, nx, ny, nz, x, y - 1, z), v0, ld(W, nx, ny, nz, x, y + 1, z),
                              ld(W, nx, ny, nz, x, y + 2, z));
        const T d2z = d2_own(ld(W, nx, ny, nz, x, y, z - 1), v0, ld(W, nx, ny, nz, x, y, z + 1));
        const T F = momentum(d2x, d2y, d2z, pc, ld(P, nx, ny, nz, x, y, z - 1), nu, axis == 2 ? drive : T(0));
        Wo[t] = (c & kSolidBit) ? T(0) : fma(dt, F, v0);
    }
}

template <typename T>
__global__ void k_simple_pres(int nx, int ny, int nz, const T *__restrict__ U, const T *__restrict__ V,
                              const T *__restrict__ W, const T *__restrict__ P, T *__restrict__ Po, T c2dt)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int x = (int)(t % nx), y = (int)((t / nx) % ny), z = (int)(t / ((int64_t)nx * ny));
    const T d = divergence(U[t], ld(U, nx, ny, nz, x + 1, y, z), V[t], ld(V, nx, ny, nz, x, y + 1, z), W[t],
                           ld(W, nx, ny, nz, x, y, z + 1));
    Po[t] = fma(-c2dt, d, P[t]);
}

template <typename T>
static hipError_t simple_sweep_t(int nx, int ny, int nz, int axis, const uint32_t *codes, const void *const in[4],
                                 void *const out[4], double nu, double dt, double c2dt, double drive, hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL(k_simple_vel<T>, dim3(grid1d(n, 256)), dim3(256), 0, s, nx, ny, nz, axis, codes,
                       (const T *)in[0], (const T *)in[1], (const T *)in[2], (const T *)in[3], (T *)out[0],
                       (T *)out[1], (T *)out[2], (T)nu, (T)dt, (T)drive);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_simple_pres<T>, dim3(grid1d(n, 256)), dim3(256), 0, s, nx, ny, nz, (const T *)out[0],
                       (const T *)out[1], (const T *)out[2], (const T *)in[3], (T *)out[3], (T)c2dt);
    return hipGetLastError();
}

hipError_t launch_simple_sweep(Prec prec, int nx, int ny, int nz, int axis, const uint32_t *codes,
                               const void *const in[4], void *const out[4], double nu, double dt, double c2dt,
                               double drive, hipStream_t s)
{
    return prec == kF64 ? simple_sweep_t<double>(nx, ny, nz, axis, codes, in, out, nu, dt, c2dt, drive, s)
                        : simple_sweep_t<float>(nx, ny, nz, axis, codes, in, out, nu, dt, c2dt, drive, s);
}

// ============================================================== state sums
//
// S_F, S_D and the face sums of a state (v, p), one thread per cell, FP64
// accumulation, per-block partials reduced afterwards in a fixed order.

constexpr int kSumsBlock = 256;
constexpr int64_t kSumsMaxBlocks = 8192;

int64_t state_sums_blocks(int64_t n)
{
    int64_t b = (n + kSumsBlock - 1) / kSumsBlock;
    return b < kSumsMaxBlocks ? b : kSumsMaxBlocks;
}

template <typename T>
__global__ void k_state_sums(int nx, int ny, int nz, int axis, const uint32_t *__restrict__ codes,
                             const T *__restrict__ U, const T *__restrict__ V, const T *__restrict__ W,
                             const T *__restrict__ P, T nu, T drive, double *__restrict__ partials)
{
    __shared__ double scratch[kNumSums * (kSumsBlock / 64)];
    const int64_t n = (int64_t)nx * ny * nz;
    double acc[kNumSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(t % nx), y = (int)((t / nx) % ny), z = (int)(t / ((int64_t)nx * ny));
        const uint32_t code = codes[t];
        const T pc = P[t];
        const T* F3[3] = {U, V, W};
        for (int k = 0; k < 3; ++k) {
            const uint32_t c = code >> (kCodeBits * k);
            const T *f = F3[k];
            const T v0 = f[t];
            acc[2 + k] += (double)v0;
            if (c & kSolidBit) continue;
            T d2[3];
            const int i1 = (k == 0) ? 1 : 0;  // first perpendicular axis
            for (int i = 0; i < 3; ++i) {
                int q[3] = {x, y, z};
                auto at = [&](int d) {
                    int r[3] = {q[0], q[1], q[2]};
                    r[i] += d;
                    return ld(f, nx, ny, nz, r[0], r[1], r[2]);
                };
                if (i == k) d2[i] = d2_own(at(-1), v0, at(1));
                else {
                    const int sh = (i == i1) ? 0 : 3;
                    d2[i] = d2_perp(coef_of_code<T>((c >> sh) & 7), at(-2), at(-1), v0, at(1), at(2));
                }
            }
            int q[3] = {x, y, z};
            q[k] -= 1;
            const T pm = ld(P, nx, ny, nz, q[0], q[1], q[2]);
            const T F = momentum(d2[0], d2[1], d2[2], pc, pm, nu, k == axis ? drive : T(0));
            acc[0] += (double)F * (double)F;
        }
        const T d = divergence(U[t], ld(U, nx, ny, nz, x + 1, y, z), V[t], ld(V, nx, ny, nz, x, y + 1, z), W[t],
                               ld(W, nx, ny, nz, x, y, z + 1));
        const double nd = (double)(nu * d);
        acc[1] += nd * nd;
    }
    block_sums(acc, scratch, partials + (int64_t)blockIdx.x * kNumSums);
}

hipError_t launch_state_sums(Prec prec, int nx, int ny, int nz, int axis, const uint32_t *codes,
                             const void *const st[4], double nu, double drive, double *partials, int64_t *nblocks,
                             hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t nb = state_sums_blocks(n);
    *nblocks = nb;
    if (prec == kF64)
        hipLaunchKernelGGL(k_state_sums<double>, dim3((unsigned)nb), dim3(kSumsBlock), 0, s, nx, ny, nz, axis,
                           codes, (const double *)st[0], (const double *)st[1], (const double *)st[2],
                           (const double *)st[3], nu, drive, partials);
    else
        hipLaunchKernelGGL(k_state_sums<float>, dim3((unsigned)nb), dim3(kSumsBlock), 0, s, nx, ny, nz, axis,
                           codes, (const float *)st[0], (const float *)st[1], (const float *)st[2],
                           (const float *)st[3], (float)nu, (float)drive, partials);
    return hipGetLastError();
}

}  // namespace ps
