// Stencil-code formats of the porestokes library: the 32-bit per-cell word and
// its 16-bit packed form.  Plain constexpr C++ (host and device), so that the
// packing can be checked exhaustively by a host program.
#pragma once

#include <stdint.h>

namespace ps {

// ---------------------------------------------------------------- face codes
//
// Per cell a uint32 holds, for component k at bit offset 8k:
//   bits 0-2  stencil code along the first perpendicular axis
//   bits 3-5  stencil code along the second perpendicular axis
//   bit  6    face solid
// Perpendicular axes in order: u -> (y, z), v -> (x, z), w -> (x, y).
// A 3-bit stencil code is L | R << 1 | F << 2 (App. B neighbourhood cases):
//   L, R  the same-component face at offset -1 / +1 is solid: a wall half a
//         voxel away (§4, no-slip at voxel faces);
//   F     only one of L, R is set and the face two steps away on the open
//         side is solid: a second wall 3/2 voxels away.
constexpr int kCodeBits = 8;
constexpr uint32_t kSolidBit = 1u << 6;

// ---------------------------------------------------------------- packed codes
//
// The solver keeps the codes in 16 bits per cell (half the bytes a sweep reads
// for them).  A component's 7-bit field takes one of 37 values: a solid face,
// whose stencil codes no kernel uses, or a fluid face with two stencil codes,
// each one of the six that occur (0, L, R, L+R, L+F, R+F: F needs exactly one
// of L, R).  Component index: 36 for a solid face, else 6 r1 + r2 with r the
// rank of the stencil code in (0, 1, 2, 3, 5, 6).  The packed code is
// i_u + 37 i_v + 37^2 i_w < 37^3 = 50653.  Unpacking gives the 32-bit form
// above, with zero stencil codes on solid faces.
constexpr uint32_t kPackBase = 37, kPackSolid = 36, kPackUV = kPackBase * kPackBase;

constexpr uint32_t pack_component(uint32_t f7)
{
    if (f7 & kSolidBit) return kPackSolid;
    const uint32_t c1 = f7 & 7, c2 = (f7 >> 3) & 7;
    return (c1 < 4 ? c1 : c1 - 1) * 6 + (c2 < 4 ? c2 : c2 - 1);
}

constexpr uint32_t unpack_component(uint32_t i)
{
    if (i == kPackSolid) return kSolidBit;
    const uint32_t r1 = i / 6, r2 = i % 6;
    return (r1 < 4 ? r1 : r1 + 1) | (r2 < 4 ? r2 : r2 + 1) << 3;
}

constexpr uint16_t pack_code(uint32_t word)
{
    return (uint16_t)(pack_component(word & 0x7f) +
                      kPackBase * (pack_component((word >> kCodeBits) & 0x7f) +
                                   kPackBase * pack_component((word >> (2 * kCodeBits)) & 0x7f)));
}

constexpr uint32_t unpack_code(uint32_t p)
{
    const uint32_t iw = p / kPackUV, r = p - iw * kPackUV, iv = r / kPackBase, iu = r - iv * kPackBase;
    return unpack_component(iu) | unpack_component(iv) << kCodeBits | unpack_component(iw) << (2 * kCodeBits);
}

}  // namespace ps
