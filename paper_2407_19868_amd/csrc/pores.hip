// Pore-space connectivity on the GPU: connected components of the pore
// voxels (6-connectivity, periodic), optionally with the periodic connection
// across one axis cut, and the pieces the host needs to decide which
// components wind around the domain (percolate).  Pre-processing of §5.1
// (elimination of disconnected pore space; the solver assumes percolation).
//
// Components are found with a lock-free union-find over the voxel indices:
// every pore voxel starts as its own root, each face-adjacent pore pair is
// united by hooking the larger root under the smaller one with a 64-bit
// compare-and-swap, so a root is always the smallest index of its set and the
// final labels are canonical (the smallest linear index of the component).
// Parent links only ever decrease and always point to an ancestor, so the
// path-halving writes in find() are harmless.
//
// Every access to the parent array is an agent-scope atomic: the 8 XCDs of
// the chip have separate L2 caches, and a plain load may return a line that
// another XCD's compare-and-swap has since changed -- inside a kernel and, as
// measured, into the next one (labels that stopped at a node hooked away
// meanwhile).  Agent-scope loads and stores are coherent across the XCDs; the
// kernels that read the finished labels load them the same way.
#include "kernels.h"

namespace ps {

__device__ __forceinline__ int64_t ld_par(const int64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_par(int64_t *p, int64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t cc_find(int64_t *par, int64_t x)
{
    int64_t p = ld_par(&par[x]);
    while (p != x) {
        const int64_t g = ld_par(&par[p]);
        if (g != p) st_par(&par[x], g);  // skip a level: g is an ancestor of x
        x = p;
        p = g;
    }
    return x;
}

__device__ __forceinline__ void cc_unite(int64_t *par, int64_t a, int64_t b)
{
    a = cc_find(par, a);
    b = cc_find(par, b);
    while (a != b) {
        if (a < b) {
            const int64_t t = a;
            a = b;
            b = t;
        }
        // a > b: make b the parent of a, if a is still a root
        int64_t old = a;
        if (__hip_atomic_compare_exchange_strong(&par[a], &old, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        a = cc_find(par, old);  // a was hooked meanwhile: continue from its new root
        b = cc_find(par, b);
    }
}

__global__ void k_cc_init(const uint8_t *__restrict__ mask, int64_t n, int64_t *__restrict__ par)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) st_par(&par[t], mask[t] ? -1 : t);
}

// Unite every pore voxel with its pore neighbours at -x, -y, -z (each pair
// once); `cut` (0..2) drops the periodic connection across that axis, -1 none.
__global__ void k_cc_merge(const uint8_t *__restrict__ mask, int nx, int ny, int nz, int cut, int64_t *par)
{
    const int64_t plane = (int64_t)nx * ny, n = plane * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n || mask[t]) return;
    const int x = (int)(t % nx), y = (int)((t / nx) % ny), z = (int)(t / plane);
    if (!(cut == 0 && x == 0)) {
        const int64_t nb = x == 0 ? t + nx - 1 : t - 1;
        if (!mask[nb]) cc_unite(par, t, nb);
    }
    if (!(cut == 1 && y == 0)) {
        const int64_t nb = y == 0 ? t + (int64_t)(ny - 1) * nx : t - nx;
        if (!mask[nb]) cc_unite(par, t, nb);
    }
    if (!(cut == 2 && z == 0)) {
        const int64_t nb = z == 0 ? t + (int64_t)(nz - 1) * plane : t - plane;
        if (!mask[nb]) cc_unite(par, t, nb);
    }
}

__global__ void k_cc_flatten(int64_t *par, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && ld_par(&par[t]) >= 0) st_par(&par[t], cc_find(par, t));
}

// One round of pointer jumping, lab[t] <- lab[lab[t]]; *changed = 1 if any
// label moved.  After the flatten every label is already a root, so this
// round finds nothing to do; it is the check that the labelling settled.
__global__ void k_cc_jump(int64_t *par, int64_t n, int *changed)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t l = ld_par(&par[t]);
    if (l < 0) return;
    const int64_t ll = ld_par(&par[l]);
    if (ll != l) {
        st_par(&par[t], ll);
        __hip_atomic_store(changed, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// For each cell of the boundary plane of axis j: the labels (of a labelling
// with axis j cut) of the pore voxel at coordinate n_j - 1 and of the one at 0
// that the periodic connection joins, or -1, -1.
__global__ void k_cc_cross(const uint8_t *__restrict__ mask, int nx, int ny, int nz, int j,
                           const int64_t *__restrict__ lab, int64_t *__restrict__ pairs)
{
    const int64_t plane = (int64_t)nx * ny;
    const int n[3] = {nx, ny, nz};
    const int64_t stride[3] = {1, nx, plane};
    const int a = j == 0 ? 1 : 0, b = j == 2 ? 1 : 2;  // the two other axes
    const int64_t cells = (int64_t)n[a] * n[b];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cells) return;
    const int ca = (int)(i % n[a]), cb = (int)(i / n[a]);
    const int64_t s = ca * stride[a] + cb * stride[b];
    const int64_t r = s + (int64_t)(n[j] - 1) * stride[j];
    const bool both = !mask[s] && !mask[r];
    pairs[2 * i] = both ? ld_par(&lab[r]) : -1;
    pairs[2 * i + 1] = both ? ld_par(&lab[s]) : -1;
}

__global__ void k_gather_i64(const int64_t *__restrict__ src, const int64_t *__restrict__ idx, int64_t m,
                             int64_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] = ld_par(&src[idx[i]]);
}

// lflag[lab[i]] |= bit for a list of distinct labels (one thread per label).
__global__ void k_flag_labels(const int64_t *__restrict__ lab, int64_t m, uint8_t bit, uint8_t *__restrict__ lflag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) lflag[lab[i]] = (uint8_t)(lflag[lab[i]] | bit);
}

__global__ void k_flow_bits(const int64_t *__restrict__ lab, const uint8_t *__restrict__ lflag, int64_t n,
                            uint8_t *__restrict__ flow)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t l = ld_par(&lab[t]);
    flow[t] = l >= 0 ? lflag[l] : (uint8_t)0;
}

// counts: [0] pore voxels, [1] components (roots), [2 + j] voxels with flow bit j
__global__ void k_pore_counts(const int64_t *__restrict__ lab, const uint8_t *__restrict__ flow, int64_t n,
                              unsigned long long *__restrict__ counts)
{
    __shared__ unsigned long long sc[5];
    if (threadIdx.x < 5) sc[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long c[5] = {0, 0, 0, 0, 0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = ld_par(&lab[t]);
        c[0] += l >= 0;
        c[1] += l == t;
        const uint8_t f = flow[t];
        for (int j = 0; j < 3; ++j) c[2 + j] += (f >> j) & 1u;
    }
    for (int i = 0; i < 5; ++i) atomicAdd(&sc[i], c[i]);
    __syncthreads();
    if (threadIdx.x < 5) atomicAdd(&counts[threadIdx.x], sc[threadIdx.x]);
}

// cleaned[t] = 1 unless t is a pore voxel whose component winds along axis j
__global__ void k_clean_mask(const uint8_t *__restrict__ flow, int64_t n, int j, uint8_t *__restrict__ cleaned)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) cleaned[t] = ((flow[t] >> j) & 1u) ? 0 : 1;
}

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_cc_label(const uint8_t *mask, int nx, int ny, int nz, int cut, int64_t *labels, hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL(k_cc_init, dim3(blocks_for(n)), dim3(256), 0, s, mask, n, labels);
    hipLaunchKernelGGL(k_cc_merge, dim3(blocks_for(n)), dim3(256), 0, s, mask, nx, ny, nz, cut, labels);
    hipLaunchKernelGGL(k_cc_flatten, dim3(blocks_for(n)), dim3(256), 0, s, labels, n);
    return hipGetLastError();
}

hipError_t launch_cc_jump(int64_t *labels, int64_t n, int *changed, hipStream_t s)
{
    hipError_t e = hipMemsetAsync(changed, 0, sizeof(int), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cc_jump, dim3(blocks_for(n)), dim3(256), 0, s, labels, n, changed);
    return hipGetLastError();
}

hipError_t launch_cc_cross(const uint8_t *mask, int nx, int ny, int nz, int j, const int64_t *labels, int64_t *pairs,
                           hipStream_t s)
{
    const int64_t n[3] = {nx, ny, nz};
    const int64_t cells = n[0] * n[1] * n[2] / n[j];
    hipLaunchKernelGGL(k_cc_cross, dim3(blocks_for(cells)), dim3(256), 0, s, mask, nx, ny, nz, j, labels, pairs);
    return hipGetLastError();
}

hipError_t launch_gather_i64(const int64_t *src, const int64_t *idx, int64_t m, int64_t *out, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_i64, dim3(blocks_for(m)), dim3(256), 0, s, src, idx, m, out);
    return hipGetLastError();
}

hipError_t launch_flag_labels(const int64_t *lab, int64_t m, int j, uint8_t *lflag, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flag_labels, dim3(blocks_for(m)), dim3(256), 0, s, lab, m, (uint8_t)(1u << j), lflag);
    return hipGetLastError();
}

hipError_t launch_flow_bits(const int64_t *labels, const uint8_t *lflag, int64_t n, uint8_t *flow, hipStream_t s)
{
    hipLaunchKernelGGL(k_flow_bits, dim3(blocks_for(n)), dim3(256), 0, s, labels, lflag, n, flow);
    return hipGetLastError();
}

hipError_t launch_pore_counts(const int64_t *labels, const uint8_t *flow, int64_t n, unsigned long long *counts,
                              hipStream_t s)
{
    hipError_t e = hipMemsetAsync(counts, 0, 5 * sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    int64_t b = blocks_for(n);
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_pore_counts, dim3((unsigned)b), dim3(256), 0, s, labels, flow, n, counts);
    return hipGetLastError();
}

hipError_t launch_clean_mask(const uint8_t *flow, int64_t n, int j, uint8_t *cleaned, hipStream_t s)
{
    hipLaunchKernelGGL(k_clean_mask, dim3(blocks_for(n)), dim3(256), 0, s, flow, n, j, cleaned);
    return hipGetLastError();
}

}  // namespace ps
