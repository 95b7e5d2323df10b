// layout.hpp -- data layouts shared by the host library and the device
// kernels (internal; plain C++, no HIP dependency, so the host-side builders
// also compile with an ordinary C++ compiler).
#pragma once

#include <stdint.h>

namespace lbm {

// Slot value meaning "no fluid node there" (solid, or beyond a wall).  The
// compact layout holds at most 2^32 - 1 fluid nodes, so no slot index takes
// this value.
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

// Segment record of the compact layout: everything a wavefront needs to know
// about one 64-node row segment (bitmap word) to find the fluid flags and
// slots of its nodes and of their x - 1 / x + 1 neighbours.
//   bits: bit b set when node x = 64 w + b is fluid (none past the row end);
//   base: slot of the first fluid node at or after x = 64 w, so the slot of a
//         fluid node is base + popcount(bits below its bit);
//   lidx: slot of the left neighbour of the segment's first node (x = 64 w - 1,
//         or nx - 1 across a periodic x boundary), kNoSlot if it is solid or
//         beyond a wall;
//   ridx: the same for the right neighbour of the segment's last node
//         (min(64 w + 63, nx - 1) + 1, or node 0 across a periodic boundary).
// The table has (ny + 2) (nz + 2) rows of W records: rows y = -1, ny and
// z = -1, nz are halo rows, copies of the wrapped rows on periodic axes and
// empty (every node solid) behind walls, so that the 9 (3-D) or 3 (2-D) rows
// around any row are found by index arithmetic alone.  32 bytes per record:
// one scalar load each.
struct SegRec {
    uint64_t bits;
    uint32_t base;
    uint32_t lidx;
    uint32_t ridx;
    uint32_t pad0;
    uint64_t pad1;
};
static_assert(sizeof(SegRec) == 32, "segment records are 32 bytes");

// Row of the record table holding row (y, z), -1 <= y <= ny, -1 <= z <= nz.
constexpr int64_t rec_row(int y, int z, int ny) { return (int64_t)(y + 1) + (int64_t)(ny + 2) * (z + 1); }

}  // namespace lbm
