// porestokes device kernels for gfx950 (MI355X).
//
//   face_bits / face_codes  mask -> face flags and per-cell stencil codes
//                           ("Evaluate neighborhood", Algorithm 1; §4, App. B)
//   fused sweep             one HBM pass per pseudo-time step (§3, Algorithm 1)
//   simple sweep            two-pass reference of the same arithmetic
//   state sums              FP64 residual and flux sums (convergence, Darcy)
#include "common.h"
#include "kernels.h"

#include <cstring>

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

__device__ uint32_t face_code(const uint8_t *__restrict__ mask, int nx, int ny, int nz, int x, int y, int z)
{
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
    return word;
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
    codes[t] = face_code(mask, nx, ny, nz, x, y, z);
}

__global__ void k_face_codes16(const uint8_t *__restrict__ mask, int nx, int ny, int nz,
                               uint16_t *__restrict__ codes)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int x = (int)(t % nx);
    const int y = (int)((t / nx) % ny);
    const int z = (int)(t / ((int64_t)nx * ny));
    codes[t] = pack_code(face_code(mask, nx, ny, nz, x, y, z));
}

__global__ void k_counts(const uint8_t *__restrict__ mask, const uint16_t *__restrict__ codes, int64_t n,
                         unsigned long long *__restrict__ counts)
{
    __shared__ unsigned long long sc[4];
    if (threadIdx.x < 4) sc[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long c[4] = {0, 0, 0, 0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        c[0] += mask[t] != 0;
        const uint32_t w = unpack_code(codes[t]);
        for (int k = 0; k < 3; ++k) c[1 + k] += ((w >> (kCodeBits * k)) & kSolidBit) == 0;
    }
    for (int i = 0; i < 4; ++i) atomicAdd(&sc[i], c[i]);
    __syncthreads();
    if (threadIdx.x < 4) atomicAdd(&counts[threadIdx.x], sc[threadIdx.x]);
}

template <typename T>
__global__ void k_zero_solid(const uint16_t *__restrict__ codes, int64_t n, T *__restrict__ u,
                             T *__restrict__ v, T *__restrict__ w)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t c = unpack_code(codes[t]);
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

struct InstTriple {
    InstDev d[3];
};

__global__ void k_store_insts(InstTriple p, int n, InstDev *__restrict__ dst)
{
    if (threadIdx.x == 0)
        for (int i = 0; i < n; ++i) dst[i] = p.d[i];
}

hipError_t launch_store_insts(const InstDev *h, int n, InstDev *dst, hipStream_t s)
{
    if (n < 1 || n > 3) return hipErrorInvalidValue;
    InstTriple p;
    std::memset(&p, 0, sizeof p);
    for (int i = 0; i < n; ++i) p.d[i] = h[i];
    hipLaunchKernelGGL(k_store_insts, dim3(1), dim3(64), 0, s, p, n, dst);
    return hipGetLastError();
}

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

hipError_t launch_face_codes16(const uint8_t *mask, int nx, int ny, int nz, uint16_t *codes, hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL(k_face_codes16, dim3(grid1d(n, 256)), dim3(256), 0, s, mask, nx, ny, nz, codes);
    return hipGetLastError();
}

hipError_t launch_counts(const uint8_t *mask, const uint16_t *codes, int64_t n, unsigned long long *counts,
                         hipStream_t s)
{
    hipError_t e = hipMemsetAsync(counts, 0, 4 * sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_counts, dim3((unsigned)blocks), dim3(256), 0, s, mask, codes, n, counts);
    return hipGetLastError();
}

hipError_t launch_zero_solid(Prec prec, const uint16_t *codes, int64_t n, void *u, void *v, void *w,
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

// The App. B coefficients of each 3-bit code sit in LDS as (a, b, gp, gm): one
// 4-wide read per lookup (one 16-byte read in FP32, two in FP64).  The far-wall
// coefficient (-1/5, on v[+2] when the near wall is at -1, on v[-2] when it is
// at +1) is nonzero for two codes only.  Same values, same operation order as
// d2_perp: the result is bitwise the same.
template <typename T>
struct alignas(4 * sizeof(T)) Coef4 {
    T a, b, gp, gm;
};

template <typename T>
__device__ __forceinline__ T d2_perp_t4(const Coef4<T> *tab, uint32_t c, T vm2, T vm1, T v0, T vp1, T vp2)
{
    const Coef4<T> k = tab[c];
    T t = k.gm * vm2;
    t = fma(k.gp, vp2, t);
    t = fma(k.b, v0, t);
    return fma(k.a, vm1 + vp1, t);
}

template <typename T>
__device__ __forceinline__ void fill_coef4(Coef4<T> *tab, int tid)
{
    if (tid < 8) {
        const Coef<T> c8 = coef_of_code<T>(tid);
        tab[tid] = {c8.a, c8.b, c8.gp, c8.gm};
    }
}

// Packed codes in the sweeps: per component a 37-entry table in LDS gives the
// component's field of the 32-bit form, already shifted into place; unpacking
// is two divisions by constants and three table reads.  (A table indexed by
// i_u + 37 i_v would save one read but costs a short z-chunk more to fill
// than to sweep.)
constexpr int kCodeLut = 3 * (int)kPackBase;

__device__ __forceinline__ void fill_code_lut(uint32_t *lut, int tid)
{
    if (tid < kCodeLut) {
        const uint32_t k = (uint32_t)tid / kPackBase, i = (uint32_t)tid - k * kPackBase;
        lut[tid] = unpack_component(i) << (kCodeBits * k);
    }
}

// The larger table, for workgroups of 1024 threads (two fills per thread):
// the (u, v) part of the code word for each r = iu + 37 iv (1369 entries),
// then the w part for each iw (37).  One division by a constant and two
// reads decode a code, against two divisions (one of them a quarter-rate
// multiply-high sequence) and three reads with the 111-entry table, which
// stays with the smaller workgroups: filling 1406 entries with 256 threads
// made the latency-bound 32^3 solve slower.
constexpr int kCodeLutBig = (int)kPackUV + (int)kPackBase;

template <int NT>
__device__ __forceinline__ void fill_code_lut_big(uint32_t *lut, int tid)
{
    for (int i = tid; i < kCodeLutBig; i += NT) {
        if (i < (int)kPackUV) {
            const uint32_t iv = (uint32_t)i / kPackBase, iu = (uint32_t)i - iv * kPackBase;
            lut[i] = unpack_component(iu) | unpack_component(iv) << kCodeBits;
        } else {
            lut[i] = unpack_component((uint32_t)i - kPackUV) << (2 * kCodeBits);
        }
    }
}

__device__ __forceinline__ uint32_t lut_code_big(const uint32_t *lut, uint32_t p)
{
    const uint32_t iw = p / kPackUV, r = p - iw * kPackUV;
    return lut[r] | lut[kPackUV + iw];
}

__device__ __forceinline__ uint32_t lut_code(const uint32_t *lut, uint32_t p)
{
    const uint32_t iw = p / kPackUV, r = p - iw * kPackUV, iv = r / kPackBase, iu = r - iv * kPackBase;
    return (lut[iu] | lut[kPackBase + iv]) | lut[2 * kPackBase + iw];
}

template <bool B>
struct BoolC {
    static constexpr bool value = B;
};

// MI355X: 8 XCDs of 32 CUs; workgroup i of a dispatch goes to XCD i mod 8.
constexpr int kNumXcd = 8;
constexpr int kCusPerXcd = 32;

// ---- raw buffer access (MUBUF).  The sweeps address one z-plane of a field
// at a time: a descriptor with the plane's base (uniform, built in scalar
// registers) and the plane's byte size as its range, plus a 32-bit per-lane
// byte offset that stays fixed along the column.  An offset at or beyond the
// range reads 0 and drops a store (the hardware's range check).
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 word 3: 32-bit data format, untyped access
constexpr int kNonTemporal = 2;         // cache policy bit: nt
constexpr int kScopeAgent = 16;         // cache policy bit: sc1 (loads bypass the CU's L1)
constexpr uint32_t kOffNone = 0x80000000u;  // beyond every plane (planes hold < 2^31 bytes)
using Rsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ Rsrc rsrc_at(const void *base, int64_t off_b, uint32_t nbytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)((const char *)base + off_b), 0, (int)nbytes, kRsrcWord3);
}

template <typename T, int AUX = 0>
__device__ __forceinline__ T bload(Rsrc r, uint32_t off)
{
    if constexpr (sizeof(T) == 2)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, AUX));
    else if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
}

template <typename T, int AUX = 0>
__device__ __forceinline__ void bstore(T v, Rsrc r, uint32_t off)
{
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, off, 0, AUX);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, AUX);
}

// Byte offset of plane z (0 <= z < nz) advanced by one plane with wrap-around.
__device__ __forceinline__ int64_t next_plane(int64_t zb, int64_t plane_b, int64_t field_b)
{
    const int64_t n = zb + plane_b;
    return n == field_b ? 0 : n;
}

// Fixed pressure (InstDev::fixp): p~ is held on the cell layer x_axis = 0.  A
// thread computes p^n of its own cell and of its -x and -y neighbours; each
// is held when it lies in that layer.  For the z axis that is a property of
// the plane (uniform): the plane at byte offset 0.
struct HeldLayer {
    bool own = false, xm = false, ym = false, fixz = false;
    __device__ __forceinline__ HeldLayer(const InstDev &I, int gx, int gy)
    {
        if (!I.fixp) return;
        const int xw = wrap_int(gx, I.nx), yw = wrap_int(gy, I.ny);
        const int xmw = wrap_int(gx - 1, I.nx), ymw = wrap_int(gy - 1, I.ny);
        own = (I.axis == 0 && xw == 0) || (I.axis == 1 && yw == 0);
        xm = (I.axis == 0 && xmw == 0) || (I.axis == 1 && yw == 0);
        ym = (I.axis == 0 && xw == 0) || (I.axis == 1 && ymw == 0);
        fixz = I.axis == 2;
    }
    __device__ __forceinline__ bool plane(int64_t zb) const { return fixz && zb == 0; }
};

template <typename T, int TX, int TY>
struct FusedShared {
    static constexpr int PX = TX + 4, PY = TY + 4, PP = PX * PY;
    T u[2][PP];
    T v[2][PP];
    T p[2][PP];
    T w[3][PP];
    Coef4<T> tab[8];
    static constexpr bool kBig = TX * TY >= 1024;
    uint32_t lut[kBig ? kCodeLutBig : kCodeLut];
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
// One workgroup's z-chunk of one sweep: block b of the launch (instance found
// from the table), reading set `parity` ^ par_off.  first: the launch's first
// sweep (the instance's `skip` applies to it only).  LAUX: cache policy of the
// field loads (kScopeAgent in the persistent sweeps, which read what other
// CUs wrote earlier in the same launch).
template <typename T, int TX, int TY, bool RED, bool SRC, int LAUX = 0>
__device__ __forceinline__ void fused_chunk(FusedShared<T, TX, TY> &sh, const InstDev *__restrict__ insts, int ninst,
                                            int64_t b, int parity, bool first)
{
    constexpr int NT = TX * TY;
    constexpr int PX = TX + 4, PY = TY + 4;
    constexpr int NHALO = PX * PY - NT;
    static_assert(NHALO <= NT, "one halo position per thread");
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
    const int64_t plane_b = plane * (int64_t)sizeof(T), field_b = plane_b * nz;  // fields
    const int64_t plane_c = plane * 2, field_c = plane_c * nz;                   // codes
    const int eff = parity ^ I.par_off;
    const T *const Uin = (const T *)I.vel[eff][0];
    const T *const Vin = (const T *)I.vel[eff][1];
    const T *const Win = (const T *)I.vel[eff][2];
    const T *const Pin = (const T *)I.pres[eff];
    T *const Uout = (T *)I.vel[eff ^ 1][0];
    T *const Vout = (T *)I.vel[eff ^ 1][1];
    T *const Wout = (T *)I.vel[eff ^ 1][2];
    T *const Pout = (T *)I.pres[eff ^ 1];
    const uint16_t *const codes = I.codes;
    const T *const Su = (const T *)I.src[0];
    const T *const Sv = (const T *)I.src[1];
    const T *const Sw = (const T *)I.src[2];
    const T *const Sp = (const T *)I.src[3];
    const T nu = (T)I.nu, dt = (T)I.dt, c2dt = (T)I.c2dt;
    const T gu = I.axis == 0 ? (T)I.drive : T(0);
    const T gv = I.axis == 1 ? (T)I.drive : T(0);
    const T gw = I.axis == 2 ? (T)I.drive : T(0);
    const bool skip = first && I.skip != 0;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    fill_coef4(sh.tab, tid);
    if constexpr (FusedShared<T, TX, TY>::kBig)
        fill_code_lut_big<NT>(sh.lut, tid);
    else
        fill_code_lut(sh.lut, tid);

    // ---- own column (inactive threads hold the wrapped column: LDS stays periodic)
    const int gx = x0 + tx, gy = y0 + ty;
    const bool active = gx < nx && gy < ny;
    const int own = wrap_int(gy, ny) * nx + wrap_int(gx, nx);
    const HeldLayer held(I, gx, gy);
    const uint32_t own_b = (uint32_t)own * (uint32_t)sizeof(T), own_c = (uint32_t)own * 2u;
    const int cl = (ty + 2) * PX + (tx + 2);  // own position in the padded plane

    // ---- halo position of this thread in the padded plane (ring of width 2)
    const bool has_halo = tid < NHALO;
    int hlds = 0;
    uint32_t hoff_b = 0;
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
        hoff_b = (uint32_t)(wrap_int(y0 - 2 + py, ny) * nx + wrap_int(x0 - 2 + px, nx)) * (uint32_t)sizeof(T);
        has_ph = (px == 1 && py >= 2 && py <= TY + 1) || (py == 1 && px >= 2 && px <= TX + 1);
    }

    // ---- prime the registers for the prologue plane zz = z0 - 1
    T Uw[5], Vw[5], Ww[3];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const int64_t zb = (int64_t)wrap_int(z0 - 3 + j, nz) * plane_b;
        Uw[j] = bload<T, LAUX>(rsrc_at(Uin, zb, plane_b), own_b);
        Vw[j] = bload<T, LAUX>(rsrc_at(Vin, zb, plane_b), own_b);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
        Ww[j] = bload<T, LAUX>(rsrc_at(Win, (int64_t)wrap_int(z0 - 2 + j, nz) * plane_b, plane_b), own_b);
    // byte offsets of planes zz .. zz + 3 (fields) and zz + 1 (codes)
    int64_t zb0 = (int64_t)wrap_int(z0 - 1, nz) * plane_b;
    int64_t zb1 = next_plane(zb0, plane_b, field_b);
    int64_t zb2 = next_plane(zb1, plane_b, field_b);
    int64_t zb3 = next_plane(zb2, plane_b, field_b);
    int64_t zc1 = (int64_t)wrap_int(z0, nz) * plane_c;
    T pold = bload<T, LAUX>(rsrc_at(Pin, zb0, plane_b), own_b);
    uint32_t code = 0;
    T sU = T(0), sV = T(0), sW = T(0), sP = T(0);  // correction-form terms of plane zz
    T hU = T(0), hV = T(0), hW = T(0), hP = T(0);
    if (has_halo) {
        hU = bload<T, LAUX>(rsrc_at(Uin, zb0, plane_b), hoff_b);
        hV = bload<T, LAUX>(rsrc_at(Vin, zb0, plane_b), hoff_b);
        hW = bload<T, LAUX>(rsrc_at(Win, zb1, plane_b), hoff_b);
        if (has_ph) hP = bload<T, LAUX>(rsrc_at(Pin, zb0, plane_b), hoff_b);
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
    // `ahead` is false only for the chunk's last plane, which loads nothing
    // for a next one; peeling it too leaves the loop without a branch around
    // its loads and without zeroing their registers (13 of 149 vector ALU
    // instructions per FP32 step, with the larger code table).
    auto plane_step = [&](const int zz, auto body_c, auto ahead_c) __attribute__((always_inline)) {
        constexpr bool body = decltype(body_c)::value;
        constexpr bool ahead = decltype(ahead_c)::value;
        T *const su = sh.u[slot];
        T *const sv = sh.v[slot];
        T *const sp = sh.p[slot];
        T *const swc = sh.w[wc];
        T *const swn = sh.w[wn];

        // ---- stage plane zz (u, v, p) and plane zz + 1 (w)
        auto stage = [&]() __attribute__((always_inline)) {
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
        };
        // the prologue issues its loads before it stages the primed values, so
        // that both sets of loads are in flight at once (a chunk of one plane:
        // one memory round trip fewer, 32^3 solve 5.4 -> 5.2 us per sweep); in
        // the loop the staging goes first (loads first measured 0.4 % slower)
        if constexpr (body) stage();
        // ---- loads for iteration zz + 1 (planes wrap, so every address is
        // valid)
        T bU = T(0), bV = T(0), bW = T(0), bP = T(0);
        T bSu = T(0), bSv = T(0), bSw = T(0), bSp = T(0);
        uint32_t bC = 0;
        const Rsrc rU1 = rsrc_at(Uin, zb1, plane_b), rV1 = rsrc_at(Vin, zb1, plane_b);
        const Rsrc rW2 = rsrc_at(Win, zb2, plane_b), rP1 = rsrc_at(Pin, zb1, plane_b);
        if (ahead) {
            if constexpr (SRC) {
                bSu = bload<T, kNonTemporal>(rsrc_at(Su, zb1, plane_b), own_b);
                bSv = bload<T, kNonTemporal>(rsrc_at(Sv, zb1, plane_b), own_b);
                bSw = bload<T, kNonTemporal>(rsrc_at(Sw, zb1, plane_b), own_b);
                bSp = bload<T, kNonTemporal>(rsrc_at(Sp, zb1, plane_b), own_b);
            }
            bU = bload<T, LAUX>(rsrc_at(Uin, zb3, plane_b), own_b);
            bV = bload<T, LAUX>(rsrc_at(Vin, zb3, plane_b), own_b);
            bW = bload<T, LAUX>(rW2, own_b);
            bP = bload<T, LAUX>(rP1, own_b);
            bC = bload<uint16_t, kNonTemporal>(rsrc_at(codes, zc1, plane_c), own_c);
        }
        T bhU = T(0), bhV = T(0), bhW = T(0), bhP = T(0);
        if (has_halo && ahead) {
            bhU = bload<T, LAUX>(rU1, hoff_b);
            bhV = bload<T, LAUX>(rV1, hoff_b);
            bhW = bload<T, LAUX>(rW2, hoff_b);
            if (has_ph) bhP = bload<T, LAUX>(rP1, hoff_b);
        }
        if constexpr (!body) stage();
        __syncthreads();

        // ---- p^n of the own cell
        const bool hz = held.plane(zb0);
        const T dvg = divergence(Uw[2], su[cl + 1], Vw[2], sv[cl + PX], Ww[1], Ww[2]);
        const T pn = (skip || held.own || hz) ? pold : fma(-c2dt, dvg, pold);

        if constexpr (body) {
            // lanes outside the grid hold a wrapped column: they compute and
            // store exactly the values of that column's own lane
            // p^n of the -x and -y neighbours, from the staged planes
            const T dxm = divergence(su[cl - 1], Uw[2], sv[cl - 1], sv[cl - 1 + PX], swc[cl - 1], swn[cl - 1]);
            const T pxm = (skip || held.xm || hz) ? sp[cl - 1] : fma(-c2dt, dxm, sp[cl - 1]);
            const T dym = divergence(su[cl - PX], su[cl - PX + 1], sv[cl - PX], Vw[2], swc[cl - PX], swn[cl - PX]);
            const T pym = (skip || held.ym || hz) ? sp[cl - PX] : fma(-c2dt, dym, sp[cl - PX]);
            bstore<T, kNonTemporal>(SRC ? pn + sP : pn, rsrc_at(Pout, zb0, plane_b), own_b);
            // u: own axis x, across y (LDS) and z (registers)
            uint32_t word;
            if constexpr (FusedShared<T, TX, TY>::kBig)
                word = lut_code_big(sh.lut, code);
            else
                word = lut_code(sh.lut, code);
            const uint32_t cu = word;
            const T u0 = Uw[2];
            const T u_d2x = d2_own(su[cl - 1], u0, su[cl + 1]);
            const T u_d2y = d2_perp_t4(sh.tab, cu & 7, su[cl - 2 * PX], su[cl - PX], u0, su[cl + PX], su[cl + 2 * PX]);
            const T u_d2z = d2_perp_t4(sh.tab, (cu >> 3) & 7, Uw[0], Uw[1], u0, Uw[3], Uw[4]);
            const T Fu = momentum(u_d2x, u_d2y, u_d2z, pn, pxm, nu, gu);
            const bool su_ = (cu & kSolidBit) != 0;
            bstore<T, kNonTemporal>(su_ ? T(0) : (SRC ? fma(dt, Fu, u0) + sU : fma(dt, Fu, u0)),
                                    rsrc_at(Uout, zb0, plane_b), own_b);
            // v: own axis y, across x (LDS) and z (registers)
            const uint32_t cv = word >> kCodeBits;
            const T v0 = Vw[2];
            const T v_d2x = d2_perp_t4(sh.tab, cv & 7, sv[cl - 2], sv[cl - 1], v0, sv[cl + 1], sv[cl + 2]);
            const T v_d2y = d2_own(sv[cl - PX], v0, sv[cl + PX]);
            const T v_d2z = d2_perp_t4(sh.tab, (cv >> 3) & 7, Vw[0], Vw[1], v0, Vw[3], Vw[4]);
            const T Fv = momentum(v_d2x, v_d2y, v_d2z, pn, pym, nu, gv);
            const bool sv_ = (cv & kSolidBit) != 0;
            bstore<T, kNonTemporal>(sv_ ? T(0) : (SRC ? fma(dt, Fv, v0) + sV : fma(dt, Fv, v0)),
                                    rsrc_at(Vout, zb0, plane_b), own_b);
            // w: own axis z (registers), across x and y (LDS)
            const uint32_t cw = word >> (2 * kCodeBits);
            const T w0 = Ww[1];
            const T w_d2x = d2_perp_t4(sh.tab, cw & 7, swc[cl - 2], swc[cl - 1], w0, swc[cl + 1], swc[cl + 2]);
            const T w_d2y = d2_perp_t4(sh.tab, (cw >> 3) & 7, swc[cl - 2 * PX], swc[cl - PX], w0, swc[cl + PX],
                                       swc[cl + 2 * PX]);
            const T w_d2z = d2_own(Ww[0], w0, Ww[2]);
            const T Fw = momentum(w_d2x, w_d2y, w_d2z, pn, pn_prev, nu, gw);
            const bool sw_ = (cw & kSolidBit) != 0;
            bstore<T, kNonTemporal>(sw_ ? T(0) : (SRC ? fma(dt, Fw, w0) + sW : fma(dt, Fw, w0)),
                                    rsrc_at(Wout, zb0, plane_b), own_b);
            // a held cell's mass balance is not imposed: no divergence term
            if (RED && !SRC && active) {
                const double fu = su_ ? 0.0 : (double)Fu, fv = sv_ ? 0.0 : (double)Fv,
                             fw = sw_ ? 0.0 : (double)Fw;
                acc[0] += fu * fu + fv * fv + fw * fw;
                const double nd = (held.own || hz) ? 0.0 : (double)(nu * dvg);
                acc[1] += nd * nd;
            }
            if (RED && SRC && active) {
                const double fu = su_ ? 0.0 : fma((double)sU, I.rdt, (double)Fu);
                const double fv = sv_ ? 0.0 : fma((double)sV, I.rdt, (double)Fv);
                const double fw = sw_ ? 0.0 : fma((double)sW, I.rdt, (double)Fw);
                acc[0] += fu * fu + fv * fv + fw * fw;
                const double nd =
                    (held.own || hz) ? 0.0 : (double)nu * fma(-(double)sP, I.rc2dt, (double)dvg);
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
        zb0 = zb1;
        zb1 = zb2;
        zb2 = zb3;
        zb3 = next_plane(zb3, plane_b, field_b);
        zc1 = next_plane(zc1, plane_c, field_c);
        slot ^= 1;
        wc = wn;
        wn = (wn == 2) ? 0 : wn + 1;
    };
    plane_step(z0 - 1, BoolC<false>{}, BoolC<true>{});  // z1 > z0: loads for z0
    // the prologue's loads land in the registers the loop carries: complete
    // them here, or the loop head would wait as if they were still in flight
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0) expcnt(7) lgkmcnt(15)
    for (int zz = z0; zz < z1 - 1; ++zz) plane_step(zz, BoolC<true>{}, BoolC<true>{});
    plane_step(z1 - 1, BoolC<true>{}, BoolC<false>{});
    if (RED) block_sums(acc, sh.red, I.partials + lb * kNumSums);
}

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

    fused_chunk<T, TX, TY, RED, SRC>(sh, insts, ninst, b, parity, true);
}

// ============================================================== two sweeps per pass
//
// The same fused step applied twice per HBM pass (temporal blocking, T = 2):
//
//   stage 1  (v^n, p^{n-1})     -> p^n, v^{n+1}   over the workgroup's region
//   stage 2  (v^{n+1}, p^n)     -> p^{n+1}, v^{n+2}  over the region's interior
//
// The stencil of one fused step reaches two cells across the flow (App. B), so
// an output tile of OX x OY columns needs stage 1 on the tile plus a ring of two
// columns: the workgroup holds one thread per column of that (OX + 4) x (OY + 4)
// region, and its stage-1 inputs come with a further ring of two (as in the
// single-step kernel).  Along z, stage 2 trails stage 1 by two planes; the stage-1
// results of a thread's own column stay in register windows (5 planes of u and v,
// 4 of w, 3 of p^n), and the plane stage 2 works on is staged in LDS for the
// neighbours.  Only v^n, p^{n-1} and the codes are read from HBM and only
// v^{n+2}, p^{n+1} written: the bytes of one sweep for two.  Ring threads compute
// stage 1 only; each output tile repeats the stage-1 work of its ring, and each
// z-chunk the stage-1 work of four planes beyond its ends.
//
// Every value is computed by the same expressions, in the same order, as in the
// single-step kernel (the drive, the App. B table, fma placement), so two stages
// here are bitwise two launches there.  Launches of this kernel never carry the
// reduction and never skip the pressure update: the first step of a pipeline and
// the step at a convergence check run as single steps.

template <typename T, int OX, int OY>
struct Fused2Shared {
    static constexpr int SX = OX + 4, SY = OY + 4, NT = SX * SY;  // stage-1 region: one thread per column
    static constexpr int PX = SX + 4, PY = SY + 4, PP = PX * PY;  // stage-1 inputs: the region plus a ring of 2
    T u[PP];
    T v[PP];
    T p[PP];
    T w[2][PP];
    T u2[NT];  // stage-1 results of the plane stage 2 works on
    T v2[NT];
    T p2[NT];
    T w2[2][NT];
    Coef4<T> tab[8];
    uint32_t lut[kCodeLut];
};

template <typename T, int OX, int OY>
__global__ void __launch_bounds__((OX + 4) * (OY + 4))
k_fused2(const InstDev *__restrict__ insts, int ninst, int parity)
{
    using SH = Fused2Shared<T, OX, OY>;
    constexpr int SX = SH::SX, SY = SH::SY, NT = SH::NT, PX = SH::PX, PY = SH::PY;
    constexpr int NHALO = PX * PY - NT;
    static_assert(NHALO <= NT, "one halo position per thread");
    __shared__ SH sh;

    // ---- XCD-aware order: a contiguous run of tiles per XCD (its own L2), the
    // runs rotated when a plane holds 256 or more tiles (as the FP32 single-step
    // kernel); blocks are only permuted
    const int64_t nbk = gridDim.x, xcd = blockIdx.x % kNumXcd, kx = blockIdx.x / kNumXcd;
    int64_t b;
    {
        const int64_t q = nbk / kNumXcd, rem = nbk % kNumXcd;
        const int64_t qx = xcd < rem ? q + 1 : q;
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
    const int X1 = bx * OX - 2, Y1 = by * OY - 2;  // origin of the stage-1 region
    const int z0 = bz * I.zc;
    const int zend = min(z0 + I.zc, nz);
    const int64_t plane = (int64_t)nx * ny;
    const int64_t plane_b = plane * (int64_t)sizeof(T), field_b = plane_b * nz;
    const int64_t plane_c = plane * 2, field_c = plane_c * nz;
    const int eff = parity ^ I.par_off;
    const T *const Uin = (const T *)I.vel[eff][0];
    const T *const Vin = (const T *)I.vel[eff][1];
    const T *const Win = (const T *)I.vel[eff][2];
    const T *const Pin = (const T *)I.pres[eff];
    T *const Uout = (T *)I.vel[eff ^ 1][0];
    T *const Vout = (T *)I.vel[eff ^ 1][1];
    T *const Wout = (T *)I.vel[eff ^ 1][2];
    T *const Pout = (T *)I.pres[eff ^ 1];
    const uint16_t *const codes = I.codes;
    const T nu = (T)I.nu, dt = (T)I.dt, c2dt = (T)I.c2dt;
    const T gu = I.axis == 0 ? (T)I.drive : T(0);
    const T gv = I.axis == 1 ? (T)I.drive : T(0);
    const T gw = I.axis == 2 ? (T)I.drive : T(0);

    const int tid = threadIdx.x;
    const int tx = tid % SX, ty = tid / SX;
    fill_coef4(sh.tab, tid);
    fill_code_lut(sh.lut, tid);

    // ---- own column (wrapped: the region may reach across the periodic boundary)
    const bool is_out = tx >= 2 && tx < SX - 2 && ty >= 2 && ty < SY - 2;
    const int own = wrap_int(Y1 + ty, ny) * nx + wrap_int(X1 + tx, nx);
    const HeldLayer held(I, X1 + tx, Y1 + ty);
    const uint32_t own_b = (uint32_t)own * (uint32_t)sizeof(T), own_c = (uint32_t)own * 2u;
    // stores: output lanes at their column (lanes of a column beyond the grid
    // store the identical values of the wrapped column); ring lanes beyond the
    // plane, where the store is dropped, so that every step stores
    // unconditionally (a path without the stores made the compiler wait for
    // each step's stores before the next loads, see the single-step kernel)
    const uint32_t st_b = is_out ? own_b : kOffNone;
    const int cl = (ty + 2) * PX + (tx + 2);  // stage-1 position in the padded plane
    const int c2 = tid;                       // stage-2 position (ty * SX + tx)

    // ---- halo position of this thread in the padded stage-1 plane (ring of width 2)
    const bool has_halo = tid < NHALO;
    int hlds = 0;
    uint32_t hoff_b = 0;
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
        hoff_b = (uint32_t)(wrap_int(Y1 - 2 + py, ny) * nx + wrap_int(X1 - 2 + px, nx)) * (uint32_t)sizeof(T);
        has_ph = (px == 1 && py >= 2 && py <= SY + 1) || (py == 1 && px >= 2 && px <= SX + 1);
    }

    // ---- stage-1 windows, primed for the prologue plane zz = z0 - 3
    T Uw[5], Vw[5], Ww[3];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const int64_t zb = (int64_t)wrap_int(z0 - 5 + j, nz) * plane_b;
        Uw[j] = bload<T>(rsrc_at(Uin, zb, plane_b), own_b);
        Vw[j] = bload<T>(rsrc_at(Vin, zb, plane_b), own_b);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
        Ww[j] = bload<T>(rsrc_at(Win, (int64_t)wrap_int(z0 - 4 + j, nz) * plane_b, plane_b), own_b);
    int64_t zb0 = (int64_t)wrap_int(z0 - 3, nz) * plane_b;  // zz
    int64_t zb1 = next_plane(zb0, plane_b, field_b);         // zz + 1
    int64_t zb2 = next_plane(zb1, plane_b, field_b);         // zz + 2
    int64_t zb3 = next_plane(zb2, plane_b, field_b);         // zz + 3
    int64_t zc1 = (int64_t)wrap_int(z0 - 2, nz) * plane_c;  // codes of zz + 1
    int64_t zout = (int64_t)wrap_int(z0 - 1, nz) * plane_b;  // the plane of the next stage-2 step
    T pold = bload<T>(rsrc_at(Pin, zb0, plane_b), own_b);
    uint32_t code = 0;
    T hU = T(0), hV = T(0), hW = T(0), hP = T(0);
    if (has_halo) {
        hU = bload<T>(rsrc_at(Uin, zb0, plane_b), hoff_b);
        hV = bload<T>(rsrc_at(Vin, zb0, plane_b), hoff_b);
        hW = bload<T>(rsrc_at(Win, zb1, plane_b), hoff_b);
        if (has_ph) hP = bload<T>(rsrc_at(Pin, zb0, plane_b), hoff_b);
    }
    int wc = 0, wn = 1;    // stage-1 w slots of planes zz and zz + 1
    int wc2 = 0, wn2 = 1;  // stage-2 w slots of planes z2 and z2 + 1
    T pn_prev = T(0), pn_prev2 = T(0);
    // stage-1 results of the own column: u, v at zz-4..zz, w at zz-3..zz, p^n at
    // zz-2..zz, codes at zz-2..zz
    T U1[5], V1[5], W1[4], P1[3];
    uint32_t C1[3] = {0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < 5; ++j) U1[j] = V1[j] = T(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) W1[j] = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) P1[j] = T(0);

    // One stage-1 step on plane zz (body: the velocity update too); the
    // prologue plane only primes p^n.  stage1_only: no stage-2 step follows,
    // whose barrier would otherwise separate this step's LDS reads from the
    // next step's staging.
    auto stage1 = [&](const int zz, auto body_c, auto only_c) __attribute__((always_inline)) {
        constexpr bool body = decltype(body_c)::value;
        constexpr bool stage1_only = decltype(only_c)::value;
        T *const su = sh.u;
        T *const sv = sh.v;
        T *const sp = sh.p;
        T *const swc = sh.w[wc];
        T *const swn = sh.w[wn];
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
        // loads for plane zz + 1 (stage 1 runs to zend + 1)
        const bool ahead = zz + 1 <= zend + 1;
        T bU = T(0), bV = T(0), bW = T(0), bP = T(0);
        uint32_t bC = 0;
        const Rsrc rU1 = rsrc_at(Uin, zb1, plane_b), rV1 = rsrc_at(Vin, zb1, plane_b);
        const Rsrc rW2 = rsrc_at(Win, zb2, plane_b), rP1 = rsrc_at(Pin, zb1, plane_b);
        if (ahead) {
            bU = bload<T>(rsrc_at(Uin, zb3, plane_b), own_b);
            bV = bload<T>(rsrc_at(Vin, zb3, plane_b), own_b);
            bW = bload<T>(rW2, own_b);
            bP = bload<T>(rP1, own_b);
            bC = bload<uint16_t, kNonTemporal>(rsrc_at(codes, zc1, plane_c), own_c);
        }
        T bhU = T(0), bhV = T(0), bhW = T(0), bhP = T(0);
        if (has_halo && ahead) {
            bhU = bload<T>(rU1, hoff_b);
            bhV = bload<T>(rV1, hoff_b);
            bhW = bload<T>(rW2, hoff_b);
            if (has_ph) bhP = bload<T>(rP1, hoff_b);
        }
        __syncthreads();

        const bool hz = held.plane(zb0);
        const T dvg = divergence(Uw[2], su[cl + 1], Vw[2], sv[cl + PX], Ww[1], Ww[2]);
        const T pn = (held.own || hz) ? pold : fma(-c2dt, dvg, pold);
        if constexpr (body) {
            const T dxm = divergence(su[cl - 1], Uw[2], sv[cl - 1], sv[cl - 1 + PX], swc[cl - 1], swn[cl - 1]);
            const T pxm = (held.xm || hz) ? sp[cl - 1] : fma(-c2dt, dxm, sp[cl - 1]);
            const T dym = divergence(su[cl - PX], su[cl - PX + 1], sv[cl - PX], Vw[2], swc[cl - PX], swn[cl - PX]);
            const T pym = (held.ym || hz) ? sp[cl - PX] : fma(-c2dt, dym, sp[cl - PX]);
            const uint32_t word = lut_code(sh.lut, code);
            const uint32_t cu = word;
            const T u0 = Uw[2];
            const T u_d2x = d2_own(su[cl - 1], u0, su[cl + 1]);
            const T u_d2y = d2_perp_t4(sh.tab, cu & 7, su[cl - 2 * PX], su[cl - PX], u0, su[cl + PX], su[cl + 2 * PX]);
            const T u_d2z = d2_perp_t4(sh.tab, (cu >> 3) & 7, Uw[0], Uw[1], u0, Uw[3], Uw[4]);
            const T Fu = momentum(u_d2x, u_d2y, u_d2z, pn, pxm, nu, gu);
            const T u1 = (cu & kSolidBit) != 0 ? T(0) : fma(dt, Fu, u0);
            const uint32_t cv = word >> kCodeBits;
            const T v0 = Vw[2];
            const T v_d2x = d2_perp_t4(sh.tab, cv & 7, sv[cl - 2], sv[cl - 1], v0, sv[cl + 1], sv[cl + 2]);
            const T v_d2y = d2_own(sv[cl - PX], v0, sv[cl + PX]);
            const T v_d2z = d2_perp_t4(sh.tab, (cv >> 3) & 7, Vw[0], Vw[1], v0, Vw[3], Vw[4]);
            const T Fv = momentum(v_d2x, v_d2y, v_d2z, pn, pym, nu, gv);
            const T v1 = (cv & kSolidBit) != 0 ? T(0) : fma(dt, Fv, v0);
            const uint32_t cw = word >> (2 * kCodeBits);
            const T w0 = Ww[1];
            const T w_d2x = d2_perp_t4(sh.tab, cw & 7, swc[cl - 2], swc[cl - 1], w0, swc[cl + 1], swc[cl + 2]);
            const T w_d2y = d2_perp_t4(sh.tab, (cw >> 3) & 7, swc[cl - 2 * PX], swc[cl - PX], w0, swc[cl + PX],
                                       swc[cl + 2 * PX]);
            const T w_d2z = d2_own(Ww[0], w0, Ww[2]);
            const T Fw = momentum(w_d2x, w_d2y, w_d2z, pn, pn_prev, nu, gw);
            const T w1 = (cw & kSolidBit) != 0 ? T(0) : fma(dt, Fw, w0);
            // push the results of plane zz into the own-column windows
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                U1[j] = U1[j + 1];
                V1[j] = V1[j + 1];
            }
            U1[4] = u1;
            V1[4] = v1;
#pragma unroll
            for (int j = 0; j < 3; ++j) W1[j] = W1[j + 1];
            W1[3] = w1;
            P1[0] = P1[1];
            P1[1] = P1[2];
            P1[2] = pn;
            C1[0] = C1[1];
            C1[1] = C1[2];
            C1[2] = word;
        }
        if constexpr (stage1_only) __syncthreads();

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
        hU = bhU;
        hV = bhV;
        hW = bhW;
        hP = bhP;
        zb0 = zb1;
        zb1 = zb2;
        zb2 = zb3;
        zb3 = next_plane(zb3, plane_b, field_b);
        zc1 = next_plane(zc1, plane_c, field_c);
        wc = wn;
        wn ^= 1;
    };

    // One stage-2 step on the plane two below the last stage-1 plane (body:
    // the velocity update and the stores; the prologue plane primes p^{n+1}).
    auto stage2 = [&](auto body_c) __attribute__((always_inline)) {
        constexpr bool body = decltype(body_c)::value;
        T *const su = sh.u2;
        T *const sv = sh.v2;
        T *const sp = sh.p2;
        T *const swc = sh.w2[wc2];
        T *const swn = sh.w2[wn2];
        su[c2] = U1[2];
        sv[c2] = V1[2];
        sp[c2] = P1[0];
        swn[c2] = W1[2];
        __syncthreads();
        const bool hz = held.plane(zout);
        T pn = T(0);
        if (is_out) {
            const T dvg = divergence(U1[2], su[c2 + 1], V1[2], sv[c2 + SX], W1[1], W1[2]);
            pn = (held.own || hz) ? P1[0] : fma(-c2dt, dvg, P1[0]);
        }
        if constexpr (body) {
            T ru = T(0), rv = T(0), rw = T(0);
            if (is_out) {
                const T dxm = divergence(su[c2 - 1], U1[2], sv[c2 - 1], sv[c2 - 1 + SX], swc[c2 - 1], swn[c2 - 1]);
                const T pxm = (held.xm || hz) ? sp[c2 - 1] : fma(-c2dt, dxm, sp[c2 - 1]);
                const T dym =
                    divergence(su[c2 - SX], su[c2 - SX + 1], sv[c2 - SX], V1[2], swc[c2 - SX], swn[c2 - SX]);
                const T pym = (held.ym || hz) ? sp[c2 - SX] : fma(-c2dt, dym, sp[c2 - SX]);
                const uint32_t cu = C1[0];
                const T u0 = U1[2];
                const T u_d2x = d2_own(su[c2 - 1], u0, su[c2 + 1]);
                const T u_d2y =
                    d2_perp_t4(sh.tab, cu & 7, su[c2 - 2 * SX], su[c2 - SX], u0, su[c2 + SX], su[c2 + 2 * SX]);
                const T u_d2z = d2_perp_t4(sh.tab, (cu >> 3) & 7, U1[0], U1[1], u0, U1[3], U1[4]);
                const T Fu = momentum(u_d2x, u_d2y, u_d2z, pn, pxm, nu, gu);
                ru = (cu & kSolidBit) != 0 ? T(0) : fma(dt, Fu, u0);
                const uint32_t cv = cu >> kCodeBits;
                const T v0 = V1[2];
                const T v_d2x = d2_perp_t4(sh.tab, cv & 7, sv[c2 - 2], sv[c2 - 1], v0, sv[c2 + 1], sv[c2 + 2]);
                const T v_d2y = d2_own(sv[c2 - SX], v0, sv[c2 + SX]);
                const T v_d2z = d2_perp_t4(sh.tab, (cv >> 3) & 7, V1[0], V1[1], v0, V1[3], V1[4]);
                const T Fv = momentum(v_d2x, v_d2y, v_d2z, pn, pym, nu, gv);
                rv = (cv & kSolidBit) != 0 ? T(0) : fma(dt, Fv, v0);
                const uint32_t cw = cu >> (2 * kCodeBits);
                const T w0 = W1[1];
                const T w_d2x = d2_perp_t4(sh.tab, cw & 7, swc[c2 - 2], swc[c2 - 1], w0, swc[c2 + 1], swc[c2 + 2]);
                const T w_d2y = d2_perp_t4(sh.tab, (cw >> 3) & 7, swc[c2 - 2 * SX], swc[c2 - SX], w0, swc[c2 + SX],
                                           swc[c2 + 2 * SX]);
                const T w_d2z = d2_own(W1[0], w0, W1[2]);
                const T Fw = momentum(w_d2x, w_d2y, w_d2z, pn, pn_prev2, nu, gw);
                rw = (cw & kSolidBit) != 0 ? T(0) : fma(dt, Fw, w0);
            }
            bstore<T, kNonTemporal>(pn, rsrc_at(Pout, zout, plane_b), st_b);
            bstore<T, kNonTemporal>(ru, rsrc_at(Uout, zout, plane_b), st_b);
            bstore<T, kNonTemporal>(rv, rsrc_at(Vout, zout, plane_b), st_b);
            bstore<T, kNonTemporal>(rw, rsrc_at(Wout, zout, plane_b), st_b);
        }
        pn_prev2 = pn;
        zout = next_plane(zout, plane_b, field_b);
        wc2 = wn2;
        wn2 ^= 1;
    };

    // stage 1 on planes z0 - 3 (prologue) .. zend + 1; stage 2 two planes behind,
    // on z0 - 1 (prologue) .. zend - 1
    stage1(z0 - 3, BoolC<false>{}, BoolC<true>{});
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the prologue's loads are in the carried registers
    stage1(z0 - 2, BoolC<true>{}, BoolC<true>{});
    stage1(z0 - 1, BoolC<true>{}, BoolC<true>{});
    stage1(z0, BoolC<true>{}, BoolC<true>{});
    stage1(z0 + 1, BoolC<true>{}, BoolC<false>{});
    stage2(BoolC<false>{});
    // no stores since the last loads: complete them here, or the loop head would
    // wait for the stores of every step as well
    __builtin_amdgcn_s_waitcnt(0x0F70);
    for (int zz = z0 + 2; zz <= zend + 1; ++zz) {
        stage1(zz, BoolC<true>{}, BoolC<false>{});
        stage2(BoolC<true>{});
    }
}

bool fused2_tile_supported(int ox, int oy, int prec)
{
    (void)prec;
    return (ox == 64 && oy == 10) || (ox == 64 && oy == 8) || (ox == 64 && oy == 6) || (ox == 32 && oy == 24) ||
           (ox == 32 && oy == 12) || (ox == 32 && oy == 8);
}

template <typename T>
static hipError_t launch_fused2_t(int ox, int oy, const InstDev *insts, int ninst, int64_t nblocks, int parity,
                                  hipStream_t s)
{
    const dim3 grid((unsigned)nblocks);
#define PS_FUSED2_CASE(OX_, OY_)                                                                            \
    if (ox == OX_ && oy == OY_) {                                                                          \
        hipLaunchKernelGGL((k_fused2<T, OX_, OY_>), grid, dim3((OX_ + 4) * (OY_ + 4)), 0, s, insts, ninst,    \
                           parity);                                                                        \
        return hipGetLastError();                                                                          \
    }
    PS_FUSED2_CASE(64, 10)
    PS_FUSED2_CASE(64, 8)
    PS_FUSED2_CASE(64, 6)
    PS_FUSED2_CASE(32, 24)
    PS_FUSED2_CASE(32, 12)
    PS_FUSED2_CASE(32, 8)
#undef PS_FUSED2_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_fused2(Prec prec, int ox, int oy, const InstDev *insts, int ninst, int64_t nblocks, int parity,
                         hipStream_t s)
{
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (!fused2_tile_supported(ox, oy, prec)) return hipErrorInvalidValue;
    return prec == kF64 ? launch_fused2_t<double>(ox, oy, insts, ninst, nblocks, parity, s)
                        : launch_fused2_t<float>(ox, oy, insts, ninst, nblocks, parity, s);
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

// ============================================================== persistent sweeps
//
// A small instance can run a block of sweeps inside one cooperative launch on
// one XCD: instance j of the launch (j < 8) takes the workgroups with blockIdx
// mod 8 == j (the dispatcher places workgroup i on XCD i mod 8; the engine
// checks this once per context), and its workgroups meet at a barrier between
// sweeps.  On one XCD every store lands in that XCD's L2, shared by its CUs, so
// the barrier needs no L2 write-back: each workgroup completes its stores,
// counts itself in with an atomic in L2 and polls the count with atomics in L2.
// Its field loads carry the sc1 policy bit, which reads them from L2 past the
// CU's L1: plain loads after such a barrier returned stale L1 data on nearly
// every read, and an acquire fence (L1 and L2 invalidation) instead cost 12 us
// per barrier.  A barrier costs 0.7-1.1 us with 8-32 workgroups, against 3.7 us
// with 32 for one over the whole chip (whose L2s are not coherent with each
// other).  The launch saves the launch gaps of a block but keeps an instance on
// an eighth of the chip: it gains where several small instances run side by
// side and loses on a single one, so the engine uses it only when asked.

__global__ void k_zero_u32(unsigned *__restrict__ p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// Polls of a barrier wait before it gives up (each poll is an L2 atomic round
// trip, so this is tens of milliseconds against a wait of about a microsecond).
constexpr unsigned kBarrierSpins = 1u << 16;

// Barrier among the `target / round` workgroups of one XCD; the count only
// grows (target = workgroups x barriers so far).  Polling adds `zero` (a
// launch argument, 0) so that it stays an atomic.  A wait that runs out sets
// *fail and returns false: the caller leaves the kernel.
__device__ __forceinline__ bool xcd_barrier(unsigned *cnt, unsigned target, unsigned zero, int *fail)
{
    __shared__ int s_ok;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores and loads are complete
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        unsigned spins = 0;
        int ok = 1;
        while (__hip_atomic_fetch_add(cnt, zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
            if (++spins > kBarrierSpins) {
                __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// `nsweeps` sweeps of up to 8 instances, instance j on XCD j; sweep k reads set
// (parity + k) & 1.  Only the first sweep applies an instance's `skip`.
template <typename T, int TX, int TY>
__global__ void __launch_bounds__(TX *TY)
k_fused_pers(const InstDev *__restrict__ insts, int ninst, int parity, int nsweeps, unsigned *bar, unsigned zero,
             int *fail)
{
    const int j = (int)(blockIdx.x % kNumXcd);
    if (j >= ninst) return;
    const InstDev &I = insts[j];
    const int64_t lb = blockIdx.x / kNumXcd;
    if (lb >= I.nblocks) return;
    __shared__ FusedShared<T, TX, TY> sh;
    unsigned *const cnt = bar + kBarrierStride * j;
    const unsigned nb = (unsigned)I.nblocks;
    for (int k = 0; k < nsweeps; ++k) {
        fused_chunk<T, TX, TY, false, false, kScopeAgent>(sh, insts, ninst, I.blk_begin + lb, parity ^ (k & 1),
                                                          k == 0);
        if (k + 1 < nsweeps && !xcd_barrier(cnt, nb * (unsigned)(k + 1), zero, fail)) return;
    }
}

template <typename T>
static hipError_t launch_fused_pers_t(int tx, int ty, const InstDev *insts, int ninst, int64_t max_blocks, int parity,
                                      int nsweeps, unsigned *bar, int *fail, hipStream_t s)
{
    const dim3 grid((unsigned)(kNumXcd * max_blocks));
    unsigned zero = 0u;
    void *args[] = {(void *)&insts, (void *)&ninst, (void *)&parity, (void *)&nsweeps, (void *)&bar, (void *)&zero,
                    (void *)&fail};
#define PS_PERS_CASE(TX_, TY_)                                                                                    \
    if (tx == TX_ && ty == TY_)                                                                                  \
        return hipLaunchCooperativeKernel((const void *)k_fused_pers<T, TX_, TY_>, grid, dim3(TX_ * TY_), args, 0, s);
    PS_PERS_CASE(32, 16)
#undef PS_PERS_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_fused_pers(Prec prec, int tx, int ty, const InstDev *insts, int ninst, int64_t max_blocks,
                             int parity, int nsweeps, unsigned *bar, int *fail, hipStream_t s)
{
    if (ninst < 1 || ninst > kNumXcd || max_blocks < 1 || max_blocks > kPersMaxBlocks || nsweeps < 1)
        return hipErrorInvalidValue;
    if (tx != kPersTX || ty != kPersTY) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, s, bar, (int)(kNumXcd * kBarrierStride));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return prec == kF64 ? launch_fused_pers_t<double>(tx, ty, insts, ninst, max_blocks, parity, nsweeps, bar, fail, s)
                        : launch_fused_pers_t<float>(tx, ty, insts, ninst, max_blocks, parity, nsweeps, bar, fail, s);
}

// The XCD of every workgroup of a 64-workgroup launch (hardware register
// XCC_ID), for the placement check of the persistent sweeps.
__global__ void k_xcc_ids(unsigned *out)
{
    if (threadIdx.x == 0) out[blockIdx.x] = __builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11)) & 0xfu;
}

hipError_t launch_xcc_ids(unsigned *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_xcc_ids, dim3(kXccProbeBlocks), dim3(64), 0, s, out);
    return hipGetLastError();
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
__global__ void k_simple_vel(int nx, int ny, int nz, int axis, const uint16_t *__restrict__ codes,
                             const T *__restrict__ U, const T *__restrict__ V, const T *__restrict__ W,
                             const T *__restrict__ P, T *__restrict__ Uo, T *__restrict__ Vo, T *__restrict__ Wo,
                             T nu, T dt, T drive)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int x = (int)(t % nx), y = (int)((t / nx) % ny), z = (int)(t / ((int64_t)nx * ny));
    const uint32_t code = unpack_code(codes[t]);
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
__global__ void k_simple_pres(int nx, int ny, int nz, int axis, int fixp, const T *__restrict__ U,
                              const T *__restrict__ V, const T *__restrict__ W, const T *__restrict__ P,
                              T *__restrict__ Po, T c2dt)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int x = (int)(t % nx), y = (int)((t / nx) % ny), z = (int)(t / ((int64_t)nx * ny));
    const int c[3] = {x, y, z};
    const T d = divergence(U[t], ld(U, nx, ny, nz, x + 1, y, z), V[t], ld(V, nx, ny, nz, x, y + 1, z), W[t],
                           ld(W, nx, ny, nz, x, y, z + 1));
    Po[t] = (fixp && c[axis] == 0) ? P[t] : fma(-c2dt, d, P[t]);  // held layer
}

template <typename T>
static hipError_t simple_sweep_t(int nx, int ny, int nz, int axis, const uint16_t *codes, const void *const in[4],
                                 void *const out[4], double nu, double dt, double c2dt, double drive, int fixp,
                                 hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL(k_simple_vel<T>, dim3(grid1d(n, 256)), dim3(256), 0, s, nx, ny, nz, axis, codes,
                       (const T *)in[0], (const T *)in[1], (const T *)in[2], (const T *)in[3], (T *)out[0],
                       (T *)out[1], (T *)out[2], (T)nu, (T)dt, (T)drive);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_simple_pres<T>, dim3(grid1d(n, 256)), dim3(256), 0, s, nx, ny, nz, axis, fixp,
                       (const T *)out[0], (const T *)out[1], (const T *)out[2], (const T *)in[3], (T *)out[3],
                       (T)c2dt);
    return hipGetLastError();
}

hipError_t launch_simple_sweep(Prec prec, int nx, int ny, int nz, int axis, const uint16_t *codes,
                               const void *const in[4], void *const out[4], double nu, double dt, double c2dt,
                               double drive, int fixp, hipStream_t s)
{
    return prec == kF64 ? simple_sweep_t<double>(nx, ny, nz, axis, codes, in, out, nu, dt, c2dt, drive, fixp, s)
                        : simple_sweep_t<float>(nx, ny, nz, axis, codes, in, out, nu, dt, c2dt, drive, fixp, s);
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
__global__ void k_state_sums(int nx, int ny, int nz, int axis, const uint16_t *__restrict__ codes,
                             const T *__restrict__ U, const T *__restrict__ V, const T *__restrict__ W,
                             const T *__restrict__ P, T nu, T drive, int fixp, double *__restrict__ partials)
{
    __shared__ double scratch[kNumSums * (kSumsBlock / 64)];
    const int64_t n = (int64_t)nx * ny * nz;
    double acc[kNumSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(t % nx), y = (int)((t / nx) % ny), z = (int)(t / ((int64_t)nx * ny));
        const uint32_t code = unpack_code(codes[t]);
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
        const int cc[3] = {x, y, z};
        if (fixp && cc[axis] == 0) continue;  // held layer: no mass balance
        const T d = divergence(U[t], ld(U, nx, ny, nz, x + 1, y, z), V[t], ld(V, nx, ny, nz, x, y + 1, z), W[t],
                               ld(W, nx, ny, nz, x, y, z + 1));
        const double nd = (double)(nu * d);
        acc[1] += nd * nd;
    }
    block_sums(acc, scratch, partials + (int64_t)blockIdx.x * kNumSums);
}

hipError_t launch_state_sums(Prec prec, int nx, int ny, int nz, int axis, const uint16_t *codes,
                             const void *const st[4], double nu, double drive, int fixp, double *partials,
                             int64_t *nblocks, hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t nb = state_sums_blocks(n);
    *nblocks = nb;
    if (prec == kF64)
        hipLaunchKernelGGL(k_state_sums<double>, dim3((unsigned)nb), dim3(kSumsBlock), 0, s, nx, ny, nz, axis,
                           codes, (const double *)st[0], (const double *)st[1], (const double *)st[2],
                           (const double *)st[3], nu, drive, fixp, partials);
    else
        hipLaunchKernelGGL(k_state_sums<float>, dim3((unsigned)nb), dim3(kSumsBlock), 0, s, nx, ny, nz, axis,
                           codes, (const float *)st[0], (const float *)st[1], (const float *)st[2],
                           (const float *)st[3], (float)nu, (float)drive, fixp, partials);
    return hipGetLastError();
}

}  // namespace ps
