// kernels.hpp -- launch arguments shared by the device kernels and the host
// library (internal; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "collide.hpp"
#include "layout.hpp"

namespace lbm {

// Largest block of any kernel of the library (their launch bounds); the tile
// shapes the host accepts (64 to 256 threads) and the block reductions'
// shared buffers are sized by it.
constexpr int kMaxBlockThreads = 256;

// Streaming patterns.
//  PAT_AB:        read the post-collision array A by pulling (x - c_i, or the
//                 node's own opposite slot when x - c_i is solid / a wall),
//                 write post-collision values to B at x.
//  PAT_AA_PULL:   AA step on a state stored "swapped" (P_i(x) in slot
//                 opp(i) at x): pull as above from the swapped slots,
//                 collide, push P_i(x) to slot i at x + c_i (or to slot
//                 opp(i) at x when x + c_i is solid): leaves streamed,
//                 pre-collision values in natural slots.
//  PAT_AA_LOCAL:  AA step on a streamed state in natural slots: read slot i
//                 at x, collide, write P_i(x) to slot opp(i) at x.
enum { PAT_AB = 0, PAT_AA_PULL = 1, PAT_AA_LOCAL = 2 };
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_F16 = 2 };

// Per-block monitor partial sums (doubles, fixed order).  MP_DU2 and MP_U2
// are the sums of |u - u_prev|^2 and |u|^2 behind the convergence residual,
// u_prev being the output velocity at the previous fused monitor step.
enum {
    MP_UX = 0, MP_UY, MP_UZ, MP_MASS, MP_UMAX, MP_UNYIELDED, MP_FALLBACK, MP_NONFINITE, MP_FLUID,
    MP_DU2, MP_U2, MP_DUMAX, MP_COUNT
};
// partials combine by max for these entries and by addition for the others
__host__ __device__ constexpr bool mp_is_max(int k) { return k == MP_UMAX || k == MP_DUMAX; }

// Population storage layouts.
//  LAYOUT_DENSE:   every node has a slot; slot (i, n) at i*S + n with S = N;
//                  solid mask as one byte per node.
//  LAYOUT_COMPACT: only fluid nodes have slots, numbered in node order
//                  (x fastest); slot (i, k) at i*S + k with S = fluid count
//                  rounded up to 64 and padded off multiples of 64 KiB.
//                  The mask is a bitmap per row (y, z): W = ceil(nx/64)
//                  64-bit words per row, bit x%64 of word x/64 set for
//                  fluid, and wbase[row][word] = compact index of the first
//                  fluid node at or after x = 64*word, so k(x) = wbase +
//                  popcount(bits below x).  wstart[g] names the word holding
//                  slot 64 g (the slot kernels start their search there).
//                  recs: the same rows as segment records with halo rows
//                  (SegRec), read by the row-segment kernel.
enum { LAYOUT_COMPACT = 0, LAYOUT_DENSE = 1 };  // same values as lbm_layout

struct StepArgs {
    const void* src;       // populations read
    void* dst;             // populations written (== src for AA)
    void* tau;             // PR relaxation time (double for FP64, float otherwise), in place
    const uint8_t* mask;   // dense: 1 = solid
    const uint64_t* bits;  // compact: fluid bitmap [row][W]
    const uint32_t* wbase; // compact: [row][W]
    const uint32_t* wstart; // compact: per group of 64 slots, the word [row][W] holding its first slot
    const SegRec* recs;    // compact: segment records [(ny + 2)(nz + 2)][W] (halo rows included)
    double* partials;      // MON: MP_COUNT doubles per tile (slot kernels: per block)
    double* uprev;         // MON: output velocity of the previous fused monitor, [3][S]; overwritten
    int64_t N;             // nodes
    int64_t S;             // direction stride of the population arrays
    int64_t nfluid;        // fluid nodes (compact: slots 0 .. nfluid-1 are used)
    int64_t ngroups;       // compact: ceil(nfluid / 64), entries of wstart
    int64_t nwords;        // compact: W * ny * nz
    int W;                 // compact: words per row
    int slot_bpx;          // slot kernels: ceil(ceil(nfluid / 256) / 8), blocks per XCD
    int pull_slots;        // compact neighbour phases: 1 slot kernel, 0 row-segment kernel
    int buf_rows;          // row-segment kernel with 32-bit buffer offsets (2 S storage elements fit in 2^32 bytes)
    int nx, ny, nz;
    int per[3];
    int tx, ty, tz;        // tile shape (threads per block = tx*ty*tz)
    int ntx, nty, ntz;     // tiles per axis
    int ntiles;
    int tiles_per_xcd;     // ceil(ntiles / 8): tiles handed to each XCD as one contiguous range
    int bry, brz;          // tile order: bricks of whole rows x bry row-blocks x brz planes
    int stream_hint;       // non-temporal access where the kernel supports it (state larger than the caches)
    int fallback;          // reduced precision: FP64 redo of near-yield nodes
    float h16_scale;       // FP16: 2^-k  (h = half * w * 2^-k)
    float h16_inv;         // FP16: 2^k
    Coll<double> cd;
    Coll<float> cf;
};

// Node-range kernels (readout, monitors on demand, population IO, init).
struct NodeArgs {
    void* pdf;             // population array (AB: the current post-collision copy)
    void* tau;
    const uint8_t* mask;
    const uint64_t* bits;
    const uint32_t* wbase;
    int64_t S;             // direction stride
    int W;
    int compact;
    double* partials;      // monitors on demand
    const double* uprev;   // monitors on demand: residual against it ([3][S], read only)
    double* out;           // staging (layout depends on the kernel)
    uint8_t* out_flags;
    int64_t N, n0, count;  // nodes [n0, n0 + count)
    int nx, ny, nz;
    int per[3];
    int layout;            // 0: post-collision natural, 1: post-collision swapped (AA), 2: streamed natural (AA)
    int reduce;            // monitors: write per-block partials instead of per-node outputs
    float h16_scale, h16_inv;
    double u0[3];
    Coll<double> cd;
    Coll<float> cf;
};

// Batched sweep: many independent all-fluid domains (walls only through
// non-periodic axes) stepped together.  Each simulation is cut into work
// items of 256 nodes (runs of consecutive nodes, or 3-D tiles); a persistent
// grid walks the work list.
struct BatchSim {
    int nx, ny, nz;
    int per[3];
    int op;
    int tx, ty, tz;        // tile shape (tx*ty*tz == 256)
    int ntx, nty, ntz;
    int item0, nitems;     // this simulation's work items [item0, item0 + nitems)
    int linear;            // 1: items are runs of 256 consecutive nodes (rows wrap) instead of tiles
    int64_t N;             // nodes
    int64_t S;             // direction stride: N rounded up to a multiple of 64, so that every
                           // direction's array starts on a cache-line boundary
    int64_t off_pdf;       // element offset of the simulation's population block ([i][n], stride S)
    int64_t off_tau;       // element offset of its relaxation-time block (PR)
    int64_t off_u;         // element offset of its previous-velocity block ([3][S] doubles)
    Coll<double> cd;
    Coll<float> cf;
};

struct BatchArgs {
    const BatchSim* sims;
    const int* work;       // work item -> simulation index
    int nitems, nsims;
    void* pdf;             // arena (AA: one copy)
    void* tau;
    double* partials;      // MON: MP_COUNT per work item
    double* uprev;         // MON: previous-velocity blocks (BatchSim::off_u)
    float h16_scale, h16_inv;
    int fallback;
    int xcd_chunks;        // work-item order (k_batch_step); needs a grid that is a multiple of 8
};

hipError_t launch_step(int lat, int op, int prec, int pat, bool mon, int layout, const StepArgs& a, hipStream_t s);
template <int LAT, int PREC>
hipError_t launch_step_prec(int op, int pat, bool mon, int layout, const StepArgs& a, hipStream_t s);
template <int LAT>
hipError_t launch_batch_lattice(int prec, int pat, bool mon, const BatchArgs& a, int grid, hipStream_t s);
hipError_t launch_batch_step(int lat, int prec, int pat, bool mon, const BatchArgs& a, int grid, hipStream_t s);
hipError_t launch_batch_finalize(const BatchArgs& a, const int* sims_item0, void* records, const int64_t* counter,
                                 int64_t step, int capacity, hipStream_t s);
hipError_t launch_batch_tick(int64_t* counter, hipStream_t s);
hipError_t launch_finalize(const double* partials, int64_t nparts, void* record, int64_t step, double ntotal,
                           hipStream_t s);
hipError_t launch_finalize_ring(const double* partials, int64_t nparts, void* ring, int64_t* counter, int capacity,
                                int64_t step, double ntotal, hipStream_t s);
hipError_t launch_init(int lat, int op, int prec, const NodeArgs& a, double rho0, hipStream_t s);
// max_blocks > 0 caps the grid of a monitor reduction (the nodes are then
// walked with a grid stride); *nblocks receives the grid (partials written)
hipError_t launch_readout(int lat, int op, int prec, const NodeArgs& a, hipStream_t s, int64_t* nblocks,
                          int64_t max_blocks = 0);
hipError_t launch_pop_write(int lat, int prec, const NodeArgs& a, hipStream_t s);
hipError_t launch_pop_read(int lat, int prec, const NodeArgs& a, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s);

// Allocation-free monitors: blocks of partial sums the per-GPU scratch array
// holds, and its device address on the device of stream s.
constexpr int64_t kScratchBlocks = 2048;
hipError_t scratch_partials(hipStream_t s, double** out);

}  // namespace lbm
