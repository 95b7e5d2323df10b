// batch_impl.hpp -- the batched step: many independent all-fluid domains
// (walls only through non-periodic axes) advanced by one launch per time
// step.  Every simulation is cut into tiles of 256 nodes; a work item is one
// tile (in the AA local phase, 256 consecutive nodes), so items are equally
// sized whatever the simulation's size.  A
// persistent grid walks the work list; each item reads its simulation's
// sizes, tile shape, operator and parameters from a device table (wave-
// uniform, scalar loads), so mixed operators branch per item, not per lane.
// The node update is the same collision code as the single-domain kernels,
// so a simulation gives bitwise the same state batched or alone.
#pragma once

#include <type_traits>

#include "step_impl.hpp"

namespace lbm {

// Neighbour phase (AA pull) of one tile.
template <int LAT, int OP, int PREC, int PAT, bool MON>
__device__ __forceinline__ void batch_tile(const BatchArgs& a, const BatchSim& sm, int item)
{
    static_assert(PAT == PAT_AB || PAT == PAT_AA_PULL, "neighbour phases only");
    using L = Lattice<LAT>;
    constexpr int Q = L::Q;
    using S = typename Store<PREC>::S;
    using C = typename Store<PREC>::C;
    using T = typename Store<PREC>::T;

    const int tile = item - sm.item0;
    const int t = threadIdx.x;
    int x, y, z;
    if (sm.linear) {
        // the item is a run of 256 consecutive nodes (rows wrap)
        const int m = tile * 256 + t;
        const int r = m / sm.nx;
        x = m - r * sm.nx;
        y = r % sm.ny;
        z = r / sm.ny;
    } else {
        const int lx = t % sm.tx;
        const int lyz = t / sm.tx;
        const int ly = lyz % sm.ty;
        const int lz = lyz / sm.ty;
        const int ttx = tile % sm.ntx;
        const int trem = tile / sm.ntx;
        const int tty = trem % sm.nty;
        const int ttz = trem / sm.nty;
        x = ttx * sm.tx + lx;
        y = tty * sm.ty + ly;
        z = ttz * sm.tz + lz;
    }
    const bool active = (x < sm.nx) & (y < sm.ny) & (z < sm.nz);
    // indices inside one simulation fit 32 bits (Q * S < 2^31 is checked on
    // the host); S is the direction stride
    const int St = (int)sm.S;
    const int n = x + sm.nx * (y + sm.ny * z);
    const Coll<C>& cp = [&]() -> const Coll<C>& {
        if constexpr (PREC == PREC_F64) return sm.cd;
        else return sm.cf;
    }();

    Moments<C> mo;
    Pre<C> pr;
    bool used_fb = false;
    if (active) {
        // Offset of the neighbour one step back / forward along each axis
        // (periodic axes wrap), and wall bits: bit 0 = no neighbour at -1,
        // bit 2 = none at +1.  A direction's neighbour is n plus the sum of
        // its three axis offsets, unless one of its steps meets a wall.
        const int sy = sm.nx, sz = sm.nx * sm.ny;
        const int ox[3] = {x > 0 ? -1 : sm.nx - 1, 0, x < sm.nx - 1 ? 1 : 1 - sm.nx};
        const int oy[3] = {y > 0 ? -sy : (sm.ny - 1) * sy, 0, y < sm.ny - 1 ? sy : (1 - sm.ny) * sy};
        const int oz[3] = {z > 0 ? -sz : (sm.nz - 1) * sz, 0, z < sm.nz - 1 ? sz : (1 - sm.nz) * sz};
        const unsigned wx = sm.per[0] ? 0u : (x == 0 ? 1u : 0u) | (x == sm.nx - 1 ? 4u : 0u);
        const unsigned wy = sm.per[1] ? 0u : (y == 0 ? 1u : 0u) | (y == sm.ny - 1 ? 4u : 0u);
        const unsigned wz = sm.per[2] ? 0u : (z == 0 ? 1u : 0u) | (z == sm.nz - 1 ? 4u : 0u);
        // neighbour x + s c (s = +-1 folded into cx, cy, cz): node index or -1
        auto nb = [&](int cx, int cy, int cz) -> int {
            const bool wall = ((wx >> (cx + 1)) | (wy >> (cy + 1)) | (wz >> (cz + 1))) & 1u;
            return wall ? -1 : n + ox[cx + 1] + oy[cy + 1] + oz[cz + 1];
        };
        const S* A = (const S*)a.pdf + sm.off_pdf;
        C h[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int idx;
            const int s = nb(-L::cx[i], -L::cy[i], -L::cz[i]);
            if constexpr (PAT == PAT_AB)
                idx = s >= 0 ? i * St + s : opp(i) * St + n;
            else
                idx = s >= 0 ? opp(i) * St + s : i * St + n;
            h[i] = decode<PREC>(A[idx], L::w[i], a.h16_scale);
        }
        T* tau = (T*)a.tau + sm.off_tau;
        C tau_prev = C(0);
        if constexpr (has_tau(OP)) tau_prev = (C)tau[n];

        collide_node<LAT, OP, PREC>(h, tau_prev, a.fallback, sm.cd, cp, mo, pr, used_fb);

        S* B = (S*)a.pdf + sm.off_pdf;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int idx;
            if constexpr (PAT == PAT_AB) {
                idx = i * St + n;  // A/B is not offered for batches; kept for completeness
            } else {
                const int d = nb(L::cx[i], L::cy[i], L::cz[i]);
                idx = d >= 0 ? i * St + d : opp(i) * St + n;
            }
            B[idx] = encode<PREC>(h[i], L::w[i], a.h16_inv);
        }
        if constexpr (has_tau(OP)) tau[n] = (T)pr.tau_p;
    }
    if constexpr (MON)
        monitor_block<C>(active, mo, pr, cp, used_fb, a.partials + (int64_t)item * MP_COUNT,
                         a.uprev ? a.uprev + sm.off_u : nullptr, n, St);
}

// AA local phase of one item.  This half of the AA pair touches only the
// node's own slots, so an item names 256 consecutive nodes instead of a tile
// (a simulation has at least ceil(N / 256) items; the surplus ones are
// empty) and each direction is one contiguous run per wavefront.  Ordinary
// loads and stores: with non-temporal hints this phase measured slower.
template <int LAT, int OP, int PREC, bool MON>
__device__ __forceinline__ void batch_local(const BatchArgs& a, const BatchSim& sm, int item)
{
    using L = Lattice<LAT>;
    constexpr int Q = L::Q;
    using S = typename Store<PREC>::S;
    using C = typename Store<PREC>::C;
    using T = typename Store<PREC>::T;

    const int St = (int)sm.S;  // direction stride; Q * S < 2^31 is checked on the host
    const int n = (item - sm.item0) * 256 + (int)threadIdx.x;
    const bool active = n < (int)sm.N;
    const Coll<C>& cp = [&]() -> const Coll<C>& {
        if constexpr (PREC == PREC_F64) return sm.cd;
        else return sm.cf;
    }();

    Moments<C> mo;
    Pre<C> pr;
    bool used_fb = false;
    if (active) {
        const S* A = (const S*)a.pdf + sm.off_pdf;
        C h[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) h[i] = decode<PREC>(A[i * St + n], L::w[i], a.h16_scale);
        T* tau = (T*)a.tau + sm.off_tau;
        C tau_prev = C(0);
        if constexpr (has_tau(OP)) tau_prev = (C)tau[n];

        collide_node<LAT, OP, PREC>(h, tau_prev, a.fallback, sm.cd, cp, mo, pr, used_fb);

        S* B = (S*)a.pdf + sm.off_pdf;
#pragma unroll
        for (int i = 0; i < Q; ++i) B[opp(i) * St + n] = encode<PREC>(h[i], L::w[i], a.h16_inv);
        if constexpr (has_tau(OP)) tau[n] = (T)pr.tau_p;
    }
    if constexpr (MON)
        monitor_block<C>(active, mo, pr, cp, used_fb, a.partials + (int64_t)item * MP_COUNT,
                         a.uprev ? a.uprev + sm.off_u : nullptr, n, St);
}

// Work-item order.  xcd_chunks == 0: block b takes items b, b + G, ...
// (G = grid size).  xcd_chunks == 1 (G a multiple of 8): the items are cut
// into 8 contiguous chunks and the blocks b with b mod 8 == j, which the
// hardware places on one XCD, walk chunk j; neighbouring tiles of a
// simulation then share that XCD's L2.  Both orders visit every item once.
// FB: the FP64 redo of near-yield nodes compiled in (reduced precision with
// the fallback on); without it the kernel holds no FP64 registers.
template <int LAT, int PREC, int PAT, bool MON, bool FB>
__global__ __launch_bounds__(kMaxBlockThreads) void k_batch_step(const BatchArgs a)
{
    constexpr int F = FB ? OP_FB : 0;
    int hi = a.nitems, first = blockIdx.x, stride = gridDim.x;
    if (a.xcd_chunks) {
        const int chunk = (a.nitems + 7) >> 3;
        const int lo = (blockIdx.x & 7) * chunk;
        hi = min(a.nitems, lo + chunk);
        first = lo + (blockIdx.x >> 3);
        stride = gridDim.x >> 3;
    }
    for (int item = first; item < hi; item += stride) {
        const int sim = __builtin_amdgcn_readfirstlane(a.work[item]);
        const BatchSim& sm = a.sims[sim];
        // PR or IR (the host rejects PRI for batches: its Newton solve would
        // raise the register count of this shared kernel for every item)
        if constexpr (PAT == PAT_AA_LOCAL) {
            if (sm.op == OP_PR) batch_local<LAT, OP_PR | F, PREC, MON>(a, sm, item);
            else batch_local<LAT, OP_IR | F, PREC, MON>(a, sm, item);
        } else {
            if (sm.op == OP_PR) batch_tile<LAT, OP_PR | F, PREC, PAT, MON>(a, sm, item);
            else batch_tile<LAT, OP_IR | F, PREC, PAT, MON>(a, sm, item);
        }
        // the block reduction's LDS slots are read by thread 0 after its
        // barrier; the next item must not overwrite them before that
        if constexpr (MON) __syncthreads();
    }
}

template <int LAT>
hipError_t launch_batch_lattice(int prec, int pat, bool mon, const BatchArgs& a, int grid, hipStream_t s)
{
    auto go = [&](auto P, auto PT, auto M) {
        constexpr int PV = decltype(P)::value;
        if (PV != PREC_F64 && a.fallback)
            hipLaunchKernelGGL((k_batch_step<LAT, PV, decltype(PT)::value, decltype(M)::value, PV != PREC_F64>),
                               dim3(grid), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_batch_step<LAT, PV, decltype(PT)::value, decltype(M)::value, false>), dim3(grid),
                               dim3(256), 0, s, a);
        return hipGetLastError();
    };
    using std::integral_constant;
    auto by_mon = [&](auto P, auto PT) {
        return mon ? go(P, PT, integral_constant<bool, true>{}) : go(P, PT, integral_constant<bool, false>{});
    };
    auto by_pat = [&](auto P) {
        switch (pat) {
        case PAT_AA_PULL: return by_mon(P, integral_constant<int, PAT_AA_PULL>{});
        case PAT_AA_LOCAL: return by_mon(P, integral_constant<int, PAT_AA_LOCAL>{});
        default: return (hipError_t)hipErrorInvalidValue;
        }
    };
    switch (prec) {
    case PREC_F64: return by_pat(integral_constant<int, PREC_F64>{});
    case PREC_F32: return by_pat(integral_constant<int, PREC_F32>{});
    case PREC_F16: return by_pat(integral_constant<int, PREC_F16>{});
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm
