// Host-visible launch interface of the porestokes kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ps {

enum Prec { kF64 = 0, kF32 = 1 };

// One solve instance as seen by the batched fused sweep kernel.  The table of
// instances lives in device memory; blocks of one launch are assigned to
// instances by their [blk_begin, blk_begin + nblocks) range.
struct InstDev {
    int32_t nx, ny, nz, axis;
    int32_t tiles_x, tiles_y, tiles_z, zc;
    int64_t blk_begin, nblocks;
    const uint16_t *codes;  // packed stencil codes (pack_code)
    void *vel[2][3];     // velocity sets; sweep n reads set (n & 1), writes the other
    void *pres[2];       // pressure sets; sweep n reads p^{n-1} from (n & 1), writes p^n
    double *partials;    // kNumSums doubles per block (written when reducing)
    double nu, dt, c2dt, drive;
    int32_t par_off;     // effective parity = launch parity ^ par_off
    int32_t skip;        // 1: first sweep of a pipeline, pressure passes through
    // correction form (launch_fused_src only): per-face and per-cell terms
    // added to u, v, w and p after the update, and 1/dt, 1/(c2 dt) to fold
    // them into the residual sums
    const void *src[4];
    double rdt, rc2dt;
    int32_t fixp;        // 1: p~ held on the cell layer x_axis = 0 (fixed pressure)
    int32_t pad;
};

// Write n <= 3 table entries to device memory from the launch arguments (no
// host buffer involved).
hipError_t launch_store_insts(const InstDev *h, int n, InstDev *dst, hipStream_t s);

// Reference to one instance's block partials for the final reduction.
struct PartialRef {
    const double *partials;
    int64_t nblocks;
};

hipError_t launch_face_bits(const uint8_t *mask, int nx, int ny, int nz, uint32_t *bits,
                            hipStream_t s);
hipError_t launch_face_codes(const uint8_t *mask, int nx, int ny, int nz, uint32_t *codes,
                             hipStream_t s);
// the same codes packed to 16 bits (pack_code), the form the solver reads
hipError_t launch_face_codes16(const uint8_t *mask, int nx, int ny, int nz, uint16_t *codes,
                               hipStream_t s);
// counts (device, 4 x uint64, zeroed by the launcher): solid voxels, fluid x/y/z faces
hipError_t launch_counts(const uint8_t *mask, const uint16_t *codes, int64_t n,
                         unsigned long long *counts, hipStream_t s);
// set faces flagged solid in codes to zero
hipError_t launch_zero_solid(Prec prec, const uint16_t *codes, int64_t n, void *u, void *v, void *w,
                             hipStream_t s);
// outer walls: mask padded with solid layers to (px, py, pz) >= (nx, ny, nz); fields
// embedded into the padded grid (zero in the added layers) or extracted back
hipError_t launch_pad_mask(const uint8_t *src, int nx, int ny, int nz, uint8_t *dst, int px, int py, int pz,
                           hipStream_t s);
hipError_t launch_embed(size_t elem, const void *src, int nx, int ny, int nz, void *dst, int px, int py, int pz,
                        hipStream_t s);
hipError_t launch_extract(size_t elem, const void *src, int px, int py, void *dst, int nx, int ny, int nz,
                          hipStream_t s);
// mirroring: dst has 2 n_i voxels along every axis i with bit i of axes, the second
// half the first reflected (dst[2 n_i - 1 - c] = src[c])
hipError_t launch_mirror(const uint8_t *src, int nx, int ny, int nz, int axes, uint8_t *dst, hipStream_t s);
// elementwise conversions and copies of n values
hipError_t launch_f64_to_f32(const double *src, float *dst, int64_t n, hipStream_t s);
hipError_t launch_f32_to_f64(const float *src, double *dst, int64_t n, hipStream_t s);
// dst += (double) src
hipError_t launch_add_f32_to_f64(const float *src, double *dst, int64_t n, hipStream_t s);
// d = (float)(t - s0)
hipError_t launch_defect(const double *t, const double *s0, float *d, int64_t n, hipStream_t s);

// Fused sweep over the instances of a device table (all of precision prec).
// alone: reserve LDS so that each CU holds one workgroup (see fused_alone).
hipError_t launch_fused(Prec prec, int tile_x, int tile_y, const InstDev *insts, int ninst,
                        int64_t nblocks, int parity, int reduce, hipStream_t s,
                        bool alone = false);
// The same sweep in FP32 with the correction-form terms of InstDev::src.
hipError_t launch_fused_src(int tile_x, int tile_y, const InstDev *insts, int ninst, int64_t nblocks, int parity,
                            int reduce, hipStream_t s, bool alone = false);
// Two fused steps per launch over output tiles of ox x oy columns (workgroups
// of (ox + 4) x (oy + 4) threads); never reducing, never skipping.  The table
// entries carry the decomposition of these tiles.
// Persistent sweeps of small instances (one XCD per instance, at most
// kPersMaxBlocks workgroups each): `nsweeps` sweeps of up to 8 instances in one
// cooperative launch, instance j on the workgroups with blockIdx mod 8 == j.
// bar: kPersXcds * kBarrierStride zeroed counters (the launcher clears them);
// fail: set to 1 when a barrier wait runs out (the sweeps after it are not done).
constexpr int kPersXcds = 8;
constexpr int kPersMaxBlocks = 32;
constexpr int kBarrierStride = 64;  // uint32 per counter: one per 256-byte line
constexpr int kXccProbeBlocks = 64;
constexpr size_t kPersL2Bytes = 3u << 20;  // largest working set swept on one XCD
constexpr int kPersTX = 32, kPersTY = 16;    // tile of the persistent sweeps
hipError_t launch_fused_pers(Prec prec, int tx, int ty, const InstDev *insts, int ninst, int64_t max_blocks,
                             int parity, int nsweeps, unsigned *bar, int *fail, hipStream_t s);
// XCD (hardware XCC id) of each of kXccProbeBlocks workgroups, into out[]
hipError_t launch_xcc_ids(unsigned *out, hipStream_t s);

hipError_t launch_fused2(Prec prec, int ox, int oy, const InstDev *insts, int ninst, int64_t nblocks, int parity,
                         hipStream_t s);
bool fused2_tile_supported(int ox, int oy, int prec);
// Whether a sweep of this precision and tile over planes of tiles_per_plane
// tiles runs one workgroup per CU: FP32 1024-thread tiles on planes of at least
// 1024 tiles measured 5-8 % faster so (1024^3, 1536^3) and 0 to -3.5 % on
// smaller planes (256^3 to 768^3, 1024 x 512 slabs).
bool fused_alone(Prec prec, int tx, int ty, int64_t tiles_per_plane);
bool fused_tile_supported(int tile_x, int tile_y, int prec);

// Final deterministic reduction: out[i * kNumSums + j] = sum over blocks of refs[i].
hipError_t launch_reduce_partials(const PartialRef *refs, int ninst, double *out, hipStream_t s);

// Two-pass reference sweep (velocity, then pressure), one thread per cell;
// fixp: p~ held on the cell layer x_axis = 0.
hipError_t launch_simple_sweep(Prec prec, int nx, int ny, int nz, int axis, const uint16_t *codes,
                               const void *const in[4], void *const out[4], double nu, double dt,
                               double c2dt, double drive, int fixp, hipStream_t s);

// Residual sums of a state into partials (one row of kNumSums per block);
// returns the number of blocks used through *nblocks.
hipError_t launch_state_sums(Prec prec, int nx, int ny, int nz, int axis, const uint16_t *codes,
                             const void *const st[4], double nu, double drive, int fixp, double *partials,
                             int64_t *nblocks, hipStream_t s);
int64_t state_sums_blocks(int64_t n);

// ---- pore-space connectivity (pores.hip)
// labels[t]: smallest index of t's pore component, -1 for solid; cut = axis whose
// periodic connection is dropped, -1 for none
hipError_t launch_cc_label(const uint8_t *mask, int nx, int ny, int nz, int cut, int64_t *labels, hipStream_t s);
// one round of pointer jumping over the labels; *changed (device int) = 1 if any label moved
hipError_t launch_cc_jump(int64_t *labels, int64_t n, int *changed, hipStream_t s);
// 2 x (cells of the boundary plane of axis j) labels of the voxel pairs joined across that boundary
hipError_t launch_cc_cross(const uint8_t *mask, int nx, int ny, int nz, int j, const int64_t *labels, int64_t *pairs,
                           hipStream_t s);
hipError_t launch_gather_i64(const int64_t *src, const int64_t *idx, int64_t m, int64_t *out, hipStream_t s);
hipError_t launch_flag_labels(const int64_t *lab, int64_t m, int j, uint8_t *lflag, hipStream_t s);
hipError_t launch_flow_bits(const int64_t *labels, const uint8_t *lflag, int64_t n, uint8_t *flow, hipStream_t s);
// counts (device, 5 x uint64, zeroed by the launcher): pore voxels, components, flow voxels per axis
hipError_t launch_pore_counts(const int64_t *labels, const uint8_t *flow, int64_t n, unsigned long long *counts,
                              hipStream_t s);
hipError_t launch_clean_mask(const uint8_t *flow, int64_t n, int j, uint8_t *cleaned, hipStream_t s);

}  // namespace ps
