// Multi-block launches of the batched path: one launch runs the same step
// (same kernel instance, workgroup size and dynamic LDS) for many blocks,
// each with its own argument struct and grid.  The launch's linear grid
// holds every block's workgroups in turn, each block starting at a multiple
// of 8 (so that a block's tile index keeps the launch index's XCD); a table
// names the block of every 8 workgroups (owner), a table places each block
// (start, grid), and the blocks' argument structs follow one another at a
// stride of exactly sizeof(Args), the stride the kernel indexes them with.
//
// The lookup (multi_locate) is shared by the device (each workgroup finds
// its block and its position in that block's grid) and the host checks; the
// layout (multi_layout, multi_fill) is host code used by the batched path
// and by those checks.
#pragma once

#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <vector>

namespace pa {

struct MultiGeo {
    uint32_t start, gx, gy, gz;
};
constexpr uint32_t MULTI_NONE = 0xFFFFFFFFu;

// The block of linear workgroup w and w's position (x, y, z) in that block's
// grid of (gx, gy, gz); MULTI_NONE for a padding workgroup.
__host__ __device__ inline uint32_t multi_locate(const MultiGeo *geo, const uint16_t *owner, uint32_t w,
                                                 uint32_t *x, uint32_t *y, uint32_t *z) {
    const uint32_t i = owner[w >> 3];
    const MultiGeo g = geo[i];
    const uint32_t local = w - g.start;
    const uint32_t per_z = g.gx * g.gy;
    if (local >= per_z * g.gz) return MULTI_NONE;
    *z = local / per_z;
    const uint32_t rem = local - *z * per_z;
    *y = rem / g.gx;
    *x = rem - *y * g.gx;
    return i;
}

// One member of a multi-block launch: its grid and its argument bytes.
struct MultiMember {
    uint32_t gx, gy, gz;
    const void *args;
};

inline size_t multi_align(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Byte offsets of one launch's tables inside a table buffer, and its
// workgroup count.
struct MultiLayout {
    uint32_t total;
    size_t o_args, o_geo, o_owner, end;
};

// Lay out the tables of a launch over `members` (argument structs of
// args_size = sizeof(Args) bytes each) starting at byte `off` (rounded up to
// 16).
inline MultiLayout multi_layout(const std::vector<MultiMember> &members, size_t args_size, size_t off) {
    MultiLayout L{};
    uint32_t wgs = 0;
    for (const MultiMember &m : members) {
        wgs = (uint32_t)multi_align(wgs, 8);
        wgs += m.gx * m.gy * m.gz;
    }
    L.total = (uint32_t)multi_align(wgs, 8);
    L.o_args = multi_align(off, 16);
    L.o_geo = multi_align(L.o_args + members.size() * args_size, 16);
    L.o_owner = multi_align(L.o_geo + members.size() * sizeof(MultiGeo), 16);
    L.end = multi_align(L.o_owner + (L.total / 8) * sizeof(uint16_t), 16);
    return L;
}

// Write the tables of a laid-out launch into the buffer at `base`.
inline void multi_fill(const std::vector<MultiMember> &members, size_t args_size, const MultiLayout &L,
                       unsigned char *base) {
    MultiGeo *geo = (MultiGeo *)(base + L.o_geo);
    uint16_t *owner = (uint16_t *)(base + L.o_owner);
    uint32_t wgs = 0;
    for (size_t m = 0; m < members.size(); ++m) {
        const MultiMember &M = members[m];
        memcpy(base + L.o_args + m * args_size, M.args, args_size);
        wgs = (uint32_t)multi_align(wgs, 8);
        const uint32_t n = M.gx * M.gy * M.gz;
        geo[m] = MultiGeo{wgs, M.gx, M.gy, M.gz};
        for (uint32_t w = wgs / 8; w < (wgs + n + 7) / 8; ++w) owner[w] = (uint16_t)m;
        wgs += n;
    }
}

}  // namespace pa
