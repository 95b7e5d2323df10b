// batch_impl.hpp -- the batched step: many independent all-fluid domains
// (walls only through non-periodic axes) advanced by one launch per time
// step.  Every simulation is cut into tiles of 256 nodes; a work item is one
// tile, so items are equally sized whatever the simulation's size.  A
// persistent grid walks the work list; each item reads its simulation's
// sizes, tile shape, operator and parameters from a device table (wave-
// uniform, scalar loads), so mixed operators branch per item, not per lane.
// The node update is the same collision code as the single-domain kernels,
// so a simulation gives bitwise the same state batched or alone.
#pragma once

#include <type_traits>

#include "step_impl.hpp"

namespace lbm {

template <int LAT, int OP, int PREC, int PAT, bool MON>
__device__ __forceinline__ void batch_tile(const BatchArgs& a, const BatchSim& sm, int item)
{
    using L = Lattice<LAT>;
    constexpr int Q = L::Q;
    using S = typename Store<PREC>::S;
    using C = typename Store<PREC>::C;
    using T = typename Store<PREC>::T;

    const int tile = item - sm.item0;
    const int t = threadIdx.x;
    const int lx = t % sm.tx;
    const int lyz = t / sm.tx;
    const int ly = lyz % sm.ty;
    const int lz = lyz / sm.ty;
    const int ttx = tile % sm.ntx;
    const int trem = tile / sm.ntx;
    const int tty = trem % sm.nty;
    const int ttz = trem / sm.nty;
    const int x = ttx * sm.tx + lx;
    const int y = tty * sm.ty + ly;
    const int z = ttz * sm.tz + lz;
    const bool active = (x < sm.nx) & (y < sm.ny) & (z < sm.nz);
    const int64_t N = sm.N;
    const int64_t n = x + (int64_t)sm.nx * (y + (int64_t)sm.ny * z);
    const Coll<C>& cp = [&]() -> const Coll<C>& {
        if constexpr (PREC == PREC_F64) return sm.cd;
        else return sm.cf;
    }();

    Moments<C> mo;
    Pre<C> pr;
    bool used_fb = false;
    if (active) {
        // neighbour x + s*c: its node index, or -1 beyond a wall face
        auto nb = [&](int cx, int cy, int cz) -> int64_t {
            int p0 = x + cx, p1 = y + cy, p2 = z + cz;
            if (p0 < 0 || p0 >= sm.nx) { if (!sm.per[0]) return -1; p0 = p0 < 0 ? p0 + sm.nx : p0 - sm.nx; }
            if (p1 < 0 || p1 >= sm.ny) { if (!sm.per[1]) return -1; p1 = p1 < 0 ? p1 + sm.ny : p1 - sm.ny; }
            if (p2 < 0 || p2 >= sm.nz) { if (!sm.per[2]) return -1; p2 = p2 < 0 ? p2 + sm.nz : p2 - sm.nz; }
            return p0 + (int64_t)sm.nx * (p1 + (int64_t)sm.ny * p2);
        };
        const S* A = (const S*)a.pdf + sm.off_pdf;
        C h[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int64_t idx;
            if constexpr (PAT == PAT_AA_LOCAL) {
                idx = (int64_t)i * N + n;
            } else {
                const int64_t s = nb(-L::cx[i], -L::cy[i], -L::cz[i]);
                if constexpr (PAT == PAT_AB)
                    idx = s >= 0 ? (int64_t)i * N + s : (int64_t)opp(i) * N + n;
                else
                    idx = s >= 0 ? (int64_t)opp(i) * N + s : (int64_t)i * N + n;
            }
            h[i] = decode<PREC>(A[idx], L::w[i], a.h16_scale);
        }
        T* tau = (T*)a.tau + sm.off_tau;
        C tau_prev = C(0);
        if constexpr (OP == OP_PR) tau_prev = (C)tau[n];

        collide_node<LAT, OP, PREC>(h, tau_prev, a.fallback, sm.cd, cp, mo, pr, used_fb);

        S* B = (S*)a.pdf + sm.off_pdf;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int64_t idx;
            if constexpr (PAT == PAT_AB) {
                idx = (int64_t)i * N + n;  // A/B is not offered for batches; kept for completeness
            } else if constexpr (PAT == PAT_AA_LOCAL) {
                idx = (int64_t)opp(i) * N + n;
            } else {
                const int64_t d = nb(L::cx[i], L::cy[i], L::cz[i]);
                idx = d >= 0 ? (int64_t)i * N + d : (int64_t)opp(i) * N + n;
            }
            B[idx] = encode<PREC>(h[i], L::w[i], a.h16_inv);
        }
        if constexpr (OP == OP_PR) tau[n] = (T)pr.tau_p;
    }
    if constexpr (MON)
        monitor_block<C>(active, mo, pr, cp, used_fb, a.partials + (int64_t)item * MP_COUNT,
                         a.uprev ? a.uprev + sm.off_u : nullptr, n, N);
}

template <int LAT, int PREC, int PAT, bool MON>
__global__ __launch_bounds__(256) void k_batch_step(const BatchArgs a)
{
    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const int sim = __builtin_amdgcn_readfirstlane(a.work[item]);
        const BatchSim& sm = a.sims[sim];
        if (sm.op == OP_PR) batch_tile<LAT, OP_PR, PREC, PAT, MON>(a, sm, item);
        else batch_tile<LAT, OP_IR, PREC, PAT, MON>(a, sm, item);
        // the block reduction's LDS slots are read by thread 0 after its
        // barrier; the next item must not overwrite them before that
        if constexpr (MON) __syncthreads();
    }
}

template <int LAT>
hipError_t launch_batch_lattice(int prec, int pat, bool mon, const BatchArgs& a, int grid, hipStream_t s)
{
    auto go = [&](auto P, auto PT, auto M) {
        hipLaunchKernelGGL((k_batch_step<LAT, decltype(P)::value, decltype(PT)::value, decltype(M)::value>),
                           dim3(grid), dim3(256), 0, s, a);
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
