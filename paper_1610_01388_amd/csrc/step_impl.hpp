// step_impl.hpp -- the fused stream-collide kernel (one time step), included
// by one translation unit per lattice so that the instantiations compile in
// parallel.
//
// One thread updates one node.  A block owns a tx*ty*tz tile; the solid mask
// of the tile plus a one-node halo is staged in LDS, so the 2Q neighbour
// tests of streaming and bounce-back are LDS reads.  Populations are SoA
// ([i][n], x fastest): for a fixed direction the lanes of a wavefront read
// and write consecutive addresses.  Block b is given tile
// (b mod 8) * tiles_per_xcd + b / 8: consecutive workgroups go to different
// XCDs, so this hands each XCD one contiguous slab of tiles and keeps the
// halo reuse between neighbouring tiles inside one XCD's L2.
#pragma once

#include "device_common.hpp"

namespace lbm {

// Collision of one node on its pre-collision deviations h (in place), with
// the FP64 redo of near-yield nodes in reduced precision.
template <int LAT, int OP, int PREC>
__device__ __forceinline__ void collide_node(typename Store<PREC>::C (&h)[Lattice<LAT>::Q],
                                             typename Store<PREC>::C tau_prev, int fallback,
                                             const Coll<double>& cd, const Coll<typename Store<PREC>::C>& cp,
                                             Moments<typename Store<PREC>::C>& mo,
                                             Pre<typename Store<PREC>::C>& pr, bool& used_fb)
{
    using C = typename Store<PREC>::C;
    constexpr int Q = Lattice<LAT>::Q;
    mo = moments<LAT>(h);
    pr = rheology<LAT, OP>(mo, cp, tau_prev);
    if constexpr (PREC != PREC_F64 && (OP & OP_FB) != 0) {
        if (fallback && pr.near_yield) {
            // FP64 from the stored values (exact in double), straight back
            // into h: no double copy of the populations is held
            const Moments<double> md = moments_as<LAT, double>(h);
            const Pre<double> pd = rheology<LAT, OP>(md, cd, (double)tau_prev);
            relax<LAT, OP>(h, md, pd, cd);
            pr.tau_p = (C)pd.tau_p;
            pr.unyielded = pd.unyielded;
            used_fb = true;
            return;
        }
    }
    relax<LAT, OP>(h, mo, pr, cp);
}

// Tile coordinates of the t-th tile in processing order.  Tiles are walked
// in bricks of whole rows (all x tiles) x bry row-blocks x brz planes, x
// fastest, then y, then z inside a brick, bricks y-major inside a z-slab of
// brz planes.  Neighbours in z are then ntx * bry tiles apart in the order,
// so a cache line that two z-adjacent tiles both touch (bounce-back reads
// and writes land in the node's own slots, which the wave of the next plane
// also streams) is still in the L2 the second time.  With one z-slab per
// XCD-contiguous range of tiles, the slab's neighbours stay on one XCD.  A
// bijection of [0, ntiles) for any bry in [1, nty], brz in [1, ntz].
__device__ __forceinline__ void tile_coords(const StepArgs& a, int t, int& ttx, int& tty, int& ttz)
{
    const int per_zb = a.ntx * a.nty * a.brz;
    const int zb = t / per_zb;
    const int u = t - zb * per_zb;
    const int bz = min(a.brz, a.ntz - zb * a.brz);
    const int per_yb = a.ntx * a.bry * bz;
    const int yb = u / per_yb;
    const int v = u - yb * per_yb;
    const int by = min(a.bry, a.nty - yb * a.bry);
    ttx = v % a.ntx;
    const int r = v / a.ntx;
    tty = yb * a.bry + r % by;
    ttz = zb * a.brz + r / by;
}

// Per-block monitor partial sums of the state the step started from.  With
// uprev set, the node's output velocity is compared with the one stored at
// the previous fused monitor (slot idx, components stride apart) and then
// replaces it.
template <class C>
__device__ __forceinline__ void monitor_block(bool active, const Moments<C>& mo, const Pre<C>& pr,
                                              const Coll<C>& cp, bool used_fb, double* dst, double* uprev,
                                              int64_t idx, int64_t stride)
{
    double v[MP_COUNT];
#pragma unroll
    for (int k = 0; k < MP_COUNT; ++k) v[k] = 0.0;
    if (active) {
        C uo[3];
        out_velocity(mo, pr, cp, uo);
        const double ux = uo[0], uy = uo[1], uz = uo[2], rho = pr.rho;
        const bool bad = !isfinite(rho) || !isfinite(ux) || !isfinite(uy) || !isfinite(uz);
        v[MP_UX] = ux;
        v[MP_UY] = uy;
        v[MP_UZ] = uz;
        v[MP_MASS] = rho;
        v[MP_UMAX] = bad ? INFINITY : sqrt(ux * ux + uy * uy + uz * uz);
        v[MP_UNYIELDED] = pr.unyielded ? 1.0 : 0.0;
        v[MP_FALLBACK] = used_fb ? 1.0 : 0.0;
        v[MP_NONFINITE] = bad ? 1.0 : 0.0;
        v[MP_FLUID] = 1.0;
        if (uprev) {
            double* up = uprev + idx;
            residual_terms(ux, uy, uz, bad, up, stride, v);
            up[0] = ux;
            up[stride] = uy;
            up[2 * stride] = uz;
        }
    }
    block_reduce_store<MP_COUNT>(v, dst);
}

template <int LAT, int OP, int PREC, int PAT, bool MON>
__global__ __launch_bounds__(kMaxBlockThreads) void k_step(const StepArgs a)
{
    using L = Lattice<LAT>;
    constexpr int Q = L::Q;
    constexpr int D = L::D;
    using S = typename Store<PREC>::S;
    using C = typename Store<PREC>::C;
    using T = typename Store<PREC>::T;
    constexpr bool PULLS = (PAT != PAT_AA_LOCAL);
    extern __shared__ uint8_t halo[];

    const int b = blockIdx.x;
    const int tile = (b & 7) * a.tiles_per_xcd + (b >> 3);
    if (tile >= a.ntiles) return;  // whole block leaves together

    const int t = threadIdx.x;
    const int lx = t % a.tx;
    const int lyz = t / a.tx;
    const int ly = lyz % a.ty;
    const int lz = lyz / a.ty;
    int ttx, tty, ttz;
    tile_coords(a, tile, ttx, tty, ttz);
    const int x = ttx * a.tx + lx;
    const int y = tty * a.ty + ly;
    const int z = ttz * a.tz + lz;
    const bool inside = (x < a.nx) & (y < a.ny) & (z < a.nz);
    const int64_t N = a.S;  // direction stride (= node count, dense layout)
    const int64_t n = x + (int64_t)a.nx * (y + (int64_t)a.ny * z);

    const int hx = a.tx + 2;
    const int hy = a.ty + 2;
    const int hc = (lx + 1) + hx * ((ly + 1) + hy * ((D == 3) ? lz + 1 : 0));
    if constexpr (PULLS) {
        const int hz = (D == 3) ? a.tz + 2 : 1;
        const int hn = hx * hy * hz;
        const int x0 = ttx * a.tx - 1, y0 = tty * a.ty - 1, z0 = (D == 3) ? ttz * a.tz - 1 : 0;
        for (int k = t; k < hn; k += blockDim.x) {
            const int kx = k % hx;
            const int kr = k / hx;
            const int ky = kr % hy;
            const int kz = kr / hy;
            bool out = false;
            const int gx = wrap_halo(x0 + kx, a.nx, a.per[0], out);
            const int gy = wrap_halo(y0 + ky, a.ny, a.per[1], out);
            const int gz = (D == 3) ? wrap_halo(z0 + kz, a.nz, a.per[2], out) : 0;
            halo[k] = out ? (uint8_t)1 : a.mask[gx + (int64_t)a.nx * (gy + (int64_t)a.ny * gz)];
        }
        __syncthreads();
    }
    bool solid = true;
    if (inside) solid = PULLS ? (halo[hc] != 0) : (a.mask[n] != 0);
    const bool active = inside && !solid;

    // wrapped neighbour coordinates (only used where the neighbour is fluid)
    const int xm = (x == 0) ? a.nx - 1 : x - 1, xp = (x == a.nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? a.ny - 1 : y - 1, yp = (y == a.ny - 1) ? 0 : y + 1;
    const int zm = (z == 0) ? a.nz - 1 : z - 1, zp = (z == a.nz - 1) ? 0 : z + 1;

    C h[Q];
    C tau_prev = C(0);
    const Coll<C>& cp = coll_of<C>(a);
    Moments<C> mo;
    Pre<C> pr;
    bool used_fb = false;
    if (active) {
        const S* A = (const S*)a.src;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int cx = L::cx[i], cy = L::cy[i], cz = L::cz[i];
            int64_t idx;
            if constexpr (PAT == PAT_AA_LOCAL) {
                idx = (int64_t)i * N + n;
            } else {
                const bool sb = halo[hc - cx - hx * (cy + hy * cz)] != 0;
                const int sx = cx == 0 ? x : (cx > 0 ? xm : xp);
                const int sy = cy == 0 ? y : (cy > 0 ? ym : yp);
                const int sz = cz == 0 ? z : (cz > 0 ? zm : zp);
                const int64_t ns = sx + (int64_t)a.nx * (sy + (int64_t)a.ny * sz);
                if constexpr (PAT == PAT_AB)
                    idx = sb ? (int64_t)opp(i) * N + n : (int64_t)i * N + ns;
                else
                    idx = sb ? (int64_t)i * N + n : (int64_t)opp(i) * N + ns;
            }
            h[i] = decode<PREC>(A[idx], L::w[i], a.h16_scale);
        }
        if constexpr (has_tau(OP)) tau_prev = (C)((const T*)a.tau)[n];

        collide_node<LAT, OP, PREC>(h, tau_prev, a.fallback, a.cd, cp, mo, pr, used_fb);

        S* B = (S*)a.dst;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int cx = L::cx[i], cy = L::cy[i], cz = L::cz[i];
            int64_t idx;
            if constexpr (PAT == PAT_AB) {
                idx = (int64_t)i * N + n;
            } else if constexpr (PAT == PAT_AA_LOCAL) {
                idx = (int64_t)opp(i) * N + n;
            } else {
                const bool sd = halo[hc + cx + hx * (cy + hy * cz)] != 0;
                const int dx = cx == 0 ? x : (cx > 0 ? xp : xm);
                const int dy = cy == 0 ? y : (cy > 0 ? yp : ym);
                const int dz = cz == 0 ? z : (cz > 0 ? zp : zm);
                const int64_t nd = dx + (int64_t)a.nx * (dy + (int64_t)a.ny * dz);
                idx = sd ? (int64_t)opp(i) * N + n : (int64_t)i * N + nd;
            }
            B[idx] = encode<PREC>(h[i], L::w[i], a.h16_inv);
        }
        if constexpr (has_tau(OP)) ((T*)a.tau)[n] = (T)pr.tau_p;
    }

    if constexpr (MON)
        monitor_block<C>(active, mo, pr, cp, used_fb, a.partials + (int64_t)tile * MP_COUNT, a.uprev, n, a.N);
}

// Compact-layout step: only fluid nodes have population slots.  A wavefront
// is one 64-node segment of one row (y, z): block = tx x ty x tz with tx = 64,
// 128 or 256, one wave per row segment.  For each of the 3 (2-D) or 9 (3-D)
// rows around it, the segment's record (SegRec: bitmap word, slot base and
// the slots of the segment's outer neighbours) is wave-uniform, one scalar
// load per row; halo rows in the record table stand for the wrapped rows of
// periodic axes and for the empty rows behind walls, so the nine loads carry
// no branch and are all in flight together.  Each lane then gets the fluid
// flag and slot of its x-1, x, x+1 neighbours in that row from the word's
// rank below the lane (mbcnt) and single-bit tests.
template <int LAT, int OP, int PREC, int PAT, bool MON>
__global__ __launch_bounds__(kMaxBlockThreads) void k_step_compact(const StepArgs a, const SegRec* __restrict__ recs)
{
    using L = Lattice<LAT>;
    constexpr int Q = L::Q;
    constexpr int D = L::D;
    using S = typename Store<PREC>::S;
    using C = typename Store<PREC>::C;
    using T = typename Store<PREC>::T;
    // SEL: neighbour addresses by selecting a 32-bit slot and one of two
    // wave-uniform array bases (no branch, fewer registers: more waves per
    // SIMD for the FP64 operators with a per-node solve or a tau field, and
    // for the reduced-precision kernels that hold the FP64 redo); otherwise
    // one 64-bit index per direction, which the compiler turns into branches
    // but which measured faster for FP64 IR and plain reduced precision.
    constexpr bool SEL = (PREC == PREC_F64 && op_base(OP) != OP_IR) || (OP & OP_FB) != 0;

    const int b = blockIdx.x;
    const int tile = (b & 7) * a.tiles_per_xcd + (b >> 3);
    if (tile >= a.ntiles) return;  // whole block leaves together

    const int lane = threadIdx.x & 63;
    // A tile is tx / 64 row segments wide (so a workgroup can hold adjacent
    // segments of one row, whose shared cache lines then meet in L2) by ty
    // rows by tz planes; wavefront wv takes segment wv % sx of row wv / sx.
    const int sx = a.tx >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ly = (wv / sx) % a.ty;
    const int lz = (wv / sx) / a.ty;
    int ttx, tty, ttz;
    tile_coords(a, tile, ttx, tty, ttz);
    const int seg = ttx * sx + wv % sx;  // row segment = bitmap word index
    const int x0 = seg * 64;
    const int x = x0 + lane;
    const int y = tty * a.ty + ly;
    const int z = ttz * a.tz + lz;
    const bool wave_in = (y < a.ny) && (z < a.nz) && (x0 < a.nx);
    const int64_t St = a.S;
    // a wave past the box edge reads the last row's records and keeps nothing
    const int yc = min(y, a.ny - 1), zc = min(z, a.nz - 1), sc = min(seg, a.W - 1);
    const uint64_t keep = wave_in ? ~0ull : 0ull;

    // Neighbourhood of node x: fluid flag of x + d (bit d of nbf, d = (dx, dy,
    // dz) in {-1,0,1}^3, index (dx+1) + 3 (dy+1) + 9 (dz+1)); for each of the
    // rows r = (dy+1) + 3 (dz+1), the compact index im[r] at x in that row (x
    // itself if fluid, else the next fluid node), and the wave-uniform indices
    // li[r] / ri[r] of the left neighbour of lane 0 and of the right
    // neighbour of the segment's last lane.  Within the segment the x-1 and
    // x+1 neighbours are im - 1 and im + [x fluid].
    uint32_t nbf = 0;
    uint32_t im[9], li[9], ri[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) im[r] = li[r] = ri[r] = 0;
    const bool last = (lane == 63) || (x == a.nx - 1);
    // the segment's last node: bits past it are zero, so the right-neighbour
    // flag of that lane can be placed there in the shifted word
    const int lastbit = min(63, a.nx - 1 - x0);
    // all record loads first (straight-line, so they are in flight together)
    uint64_t rb[9];
    uint32_t rbase[9], rl[9], rr[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        rb[r] = 0;
        rbase[r] = rl[r] = rr[r] = kNoSlot;
        if (D == 2 && r / 3 != 1) continue;
        const SegRec* rp = recs + rec_row(yc + r % 3 - 1, zc + r / 3 - 1, a.ny) * a.W + sc;
        rb[r] = rp->bits;
        rbase[r] = rp->base;
        rl[r] = rp->lidx;
        rr[r] = rp->ridx;
    }
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        if (D == 2 && r / 3 != 1) continue;
        const uint64_t mb = rb[r] & keep;
        const uint64_t lf = (wave_in && rl[r] != kNoSlot) ? 1ull : 0ull;
        const uint64_t rf = (wave_in && rr[r] != kNoSlot) ? 1ull : 0ull;
        // bit lane of lw / mb / rw: fluid flag of x - 1 / x / x + 1
        const uint64_t lw = (mb << 1) | lf;
        const uint64_t rw = (mb >> 1) | (rf << lastbit);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
        nbf |= (uint32_t)((lw >> lane) & 1u) << (3 * r + 0);
        nbf |= (uint32_t)((mb >> lane) & 1u) << (3 * r + 1);
        nbf |= (uint32_t)((rw >> lane) & 1u) << (3 * r + 2);
        im[r] = rbase[r] + rank;
        li[r] = rl[r];
        ri[r] = rr[r];
    }
    // compact index of the neighbour x + (dx, row r) (valid when it is fluid)
    auto nbi = [&](int dx, int r) -> uint32_t {
        if (dx == 0) return im[r];
        if (dx < 0) return lane > 0 ? im[r] - 1u : li[r];
        return !last ? im[r] + ((nbf >> (3 * r + 1)) & 1u) : ri[r];
    };
    constexpr int SELF = 13;
    const bool active = wave_in && ((nbf >> SELF) & 1);
    const int64_t k = im[4];

    C h[Q];
    C tau_prev = C(0);
    const Coll<C>& cp = coll_of<C>(a);
    Moments<C> mo;
    Pre<C> pr;
    bool used_fb = false;
    if (active) {
        const S* A = (const S*)a.src;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const S* p;
            if constexpr (PAT == PAT_AA_LOCAL) {
                p = A + (int64_t)i * St + k;
            } else {
                const int r = (1 - L::cy[i]) + 3 * (1 - L::cz[i]);  // row of x - c_i
                const bool fl = (nbf >> (3 * r + 1 - L::cx[i])) & 1;
                const int dn = PAT == PAT_AB ? i : opp(i), db = PAT == PAT_AB ? opp(i) : i;
                if constexpr (SEL) {
                    const uint32_t sl = fl ? nbi(-L::cx[i], r) : (uint32_t)k;
                    p = (fl ? A + dn * St : A + db * St) + sl;
                } else {
                    p = A + (fl ? (int64_t)dn * St + nbi(-L::cx[i], r) : (int64_t)db * St + k);
                }
            }
            h[i] = decode<PREC>(*p, L::w[i], a.h16_scale);
        }
        if constexpr (has_tau(OP)) tau_prev = (C)((const T*)a.tau)[k];

        collide_node<LAT, OP, PREC>(h, tau_prev, a.fallback, a.cd, cp, mo, pr, used_fb);

        if constexpr (PAT == PAT_AA_PULL) {
            // Rebuild the neighbour indices for the stores from im, nbf and the
            // wave-uniform edges instead of keeping the 27 load-side values
            // alive through the collision (register pressure sets the
            // occupancy of this kernel).  The empty asm only hides the values'
            // history from the optimiser; it emits no instruction.
#pragma unroll
            for (int r = 0; r < 9; ++r) asm volatile("" : "+v"(im[r]));
            if constexpr (SEL) asm volatile("" : "+v"(nbf));
        }
        S* B = (S*)a.dst;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            S* p;
            if constexpr (PAT == PAT_AB) {
                p = B + (int64_t)i * St + k;
            } else if constexpr (PAT == PAT_AA_LOCAL) {
                p = B + (int64_t)opp(i) * St + k;
            } else {
                const int r = (1 + L::cy[i]) + 3 * (1 + L::cz[i]);  // row of x + c_i
                const bool fl = (nbf >> (3 * r + 1 + L::cx[i])) & 1;
                if constexpr (SEL) {
                    const uint32_t sl = fl ? nbi(L::cx[i], r) : (uint32_t)k;
                    p = (fl ? B + i * St : B + opp(i) * St) + sl;
                } else {
                    p = B + (fl ? (int64_t)i * St + nbi(L::cx[i], r) : (int64_t)opp(i) * St + k);
                }
            }
            *p = encode<PREC>(h[i], L::w[i], a.h16_inv);
        }
        if constexpr (has_tau(OP)) ((T*)a.tau)[k] = (T)pr.tau_p;
    }
    if constexpr (MON)
        monitor_block<C>(active, mo, pr, cp, used_fb, a.partials + (int64_t)tile * MP_COUNT, a.uprev, k, St);
}

// Per-lane choice by a wave-uniform lane mask: bit `lane` of mask set gives
// a, clear gives b -- one v_cndmask_b32 that reads the mask straight from a
// scalar register pair (no per-lane bit extraction).
__device__ __forceinline__ uint32_t lane_pick(uint64_t mask, uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(mask));
    return r;
}

// A wave-uniform 64-bit value marked as such (kept in scalar registers).
__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Raw buffer access to population storage: a 32-bit byte offset from the
// descriptor's base, range-checked against its size (accesses past it read
// zero and write nothing).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pop_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
template <class S> __device__ __forceinline__ S buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <> __device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ __forceinline__ _Float16 buf_ld<_Float16>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
}
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void buf_st(double v, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_st(_Float16 v, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, off, 0, 0);
}

// Compact layout, neighbour phases (AA pull, A/B), row-segment waves with
// buffer addressing.  The geometry of the wave is that of k_step_compact
// (one 64-node row segment, the nine segment records), kept as lane masks:
// for each row r around the segment, bit `lane` of wl / wm / wr is the fluid
// flag of x - 1 / x / x + 1 in that row.  A population is read through the
// descriptor of its direction pair {i, opp(i)} (the two arrays a lane
// chooses between: the neighbour's slot in one, its own slot in the other),
// at a 32-bit element offset picked per lane by the fluid mask of the
// neighbour -- a select and an add per access, no branch and no 64-bit
// address arithmetic.  In the AA pull the store of direction i goes exactly
// where the load of opp(i) came from.  Needs 2 S (population stride) bytes
// of storage element below 2^32 (checked on the host; k_step_compact serves
// larger domains).
template <int LAT, int OP, int PREC, int PAT, bool MON>
__global__ __launch_bounds__(kMaxBlockThreads) void k_step_rows(const StepArgs a, const SegRec* __restrict__ recs)
{
    using L = Lattice<LAT>;
    constexpr int Q = L::Q;
    constexpr int D = L::D;
    using S = typename Store<PREC>::S;
    using C = typename Store<PREC>::C;
    using T = typename Store<PREC>::T;
    static_assert(PAT == PAT_AB || PAT == PAT_AA_PULL, "neighbour phases only");
    constexpr int SH = sizeof(S) == 8 ? 3 : sizeof(S) == 4 ? 2 : 1;
    // keep the 27 load offsets for the stores (reduced precision has the
    // registers to spare) or rebuild them after the collision (FP64)
    constexpr bool KEEP = sizeof(S) < 8;

    const int b = blockIdx.x;
    const int tile = (b & 7) * a.tiles_per_xcd + (b >> 3);
    if (tile >= a.ntiles) return;  // whole block leaves together

    const int lane = threadIdx.x & 63;
    const int sx = a.tx >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ly = (wv / sx) % a.ty;
    const int lz = (wv / sx) / a.ty;
    int ttx, tty, ttz;
    tile_coords(a, tile, ttx, tty, ttz);
    const int seg = ttx * sx + wv % sx;
    const int x0 = seg * 64;
    const int y = tty * a.ty + ly;
    const int z = ttz * a.tz + lz;
    const bool wave_in = (y < a.ny) && (z < a.nz) && (x0 < a.nx);
    const int yc = min(y, a.ny - 1), zc = min(z, a.nz - 1), sc = min(seg, a.W - 1);
    const uint64_t keep = wave_in ? ~0ull : 0ull;
    const int lastbit = min(63, a.nx - 1 - x0);

    uint64_t wl[9], wm[9], wr[9];
    uint32_t im[9], rl[9], rr[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        wl[r] = wm[r] = wr[r] = 0;
        im[r] = rl[r] = rr[r] = 0;
        if (D == 2 && r / 3 != 1) continue;
        const SegRec* rp = recs + rec_row(yc + r % 3 - 1, zc + r / 3 - 1, a.ny) * a.W + sc;
        wm[r] = rp->bits;
        im[r] = rp->base;
        rl[r] = rp->lidx;
        rr[r] = rp->ridx;
    }
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        if (D == 2 && r / 3 != 1) continue;
        const uint64_t mb = wm[r] & keep;
        const uint64_t lf = (wave_in && rl[r] != kNoSlot) ? 1ull : 0ull;
        const uint64_t rf = (wave_in && rr[r] != kNoSlot) ? 1ull : 0ull;
        wm[r] = uniform64(mb);
        wl[r] = uniform64((mb << 1) | lf);
        wr[r] = uniform64((mb >> 1) | (rf << lastbit));
        im[r] += __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
    }
    const bool active = (wm[4] >> lane) & 1;
    const uint32_t k = im[4];
    const uint32_t St = (uint32_t)a.S;
    const uint32_t pair_bytes = (uint32_t)(2 * a.S * (int64_t)sizeof(S));
    const uint64_t not_first = ~1ull;
    const uint64_t not_last = uniform64(~((1ull << 63) | (1ull << lastbit)));

    // element offset, within the descriptor of pair {i, opp(i)}, of the
    // population direction i pulls: the slot of x - c_i in array opp(i)
    // (AA) / i (A/B) when that node is fluid, else the node's own slot in
    // array i (AA) / opp(i) (A/B)
    auto load_elem = [&](int i) -> uint32_t {
        if (i == 0) return k;
        const int o = opp(i), lo = i < o ? i : o;
        const int r = (1 - L::cy[i]) + 3 * (1 - L::cz[i]);  // row of x - c_i
        const int dx = -L::cx[i];
        const int dn = PAT == PAT_AB ? i : o, db = PAT == PAT_AB ? o : i;
        uint32_t nb;  // slot of x - c_i
        if (dx == 0) nb = im[r];
        else if (dx < 0) nb = lane_pick(not_first, im[r] - 1u, rl[r]);
        else nb = lane_pick(not_last, lane_pick(wm[r], im[r] + 1u, im[r]), rr[r]);
        const uint64_t fl = dx < 0 ? wl[r] : dx == 0 ? wm[r] : wr[r];
        return lane_pick(fl, dn == lo ? nb : nb + St, db == lo ? k : k + St);
    };

    C h[Q];
    uint32_t off[KEEP ? Q : 1];
    C tau_prev = C(0);
    const Coll<C>& cp = coll_of<C>(a);
    Moments<C> mo;
    Pre<C> pr;
    bool used_fb = false;
    if (active) {
        const S* A = (const S*)a.src;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int o = opp(i), lo = i < o ? i : o;
            const uint32_t e = load_elem(i) << SH;
            if constexpr (KEEP) off[i] = e;
            h[i] = decode<PREC>(buf_ld<S>(pop_rsrc(A + (int64_t)lo * a.S, pair_bytes), e), L::w[i], a.h16_scale);
        }
        if constexpr (has_tau(OP)) tau_prev = (C)((const T*)a.tau)[k];

        collide_node<LAT, OP, PREC>(h, tau_prev, a.fallback, a.cd, cp, mo, pr, used_fb);

        if constexpr (PAT == PAT_AA_PULL && !KEEP) {
            // rebuild the offsets from im instead of holding 27 through the
            // collision; the empty asm hides im's history from the optimiser
#pragma unroll
            for (int r = 0; r < 9; ++r) asm volatile("" : "+v"(im[r]));
        }
        S* B = (S*)a.dst;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const S v = encode<PREC>(h[i], L::w[i], a.h16_inv);
            if constexpr (PAT == PAT_AB) {
                buf_st(v, pop_rsrc(B + (int64_t)i * a.S, pair_bytes / 2), k << SH);
            } else {
                const int o = opp(i), lo = i < o ? i : o;
                const uint32_t e = KEEP ? off[o] : (load_elem(o) << SH);
                buf_st(v, pop_rsrc(B + (int64_t)lo * a.S, pair_bytes), e);
            }
        }
        if constexpr (has_tau(OP)) ((T*)a.tau)[k] = (T)pr.tau_p;
    }
    if constexpr (MON)
        monitor_block<C>(active, mo, pr, cp, used_fb, a.partials + (int64_t)tile * MP_COUNT, a.uprev, k, a.S);
}

// Compact layout, AA local phase: every fluid node's streamed populations
// already sit in its own slots, so this half of the AA pair needs no
// geometry at all.  One thread per fluid slot, 256 slots per block: every
// lane is busy and each direction is one contiguous run per wavefront.
// NT: non-temporal loads and stores, for states larger than the caches
// (a cache-resident state would only lose its hits).  Monitor partials: one
// per block.
template <int LAT, int OP, int PREC, bool MON, bool NT>
__global__ __launch_bounds__(kMaxBlockThreads) void k_local_slots(const StepArgs a)
{
    using L = Lattice<LAT>;
    constexpr int Q = L::Q;
    using S = typename Store<PREC>::S;
    using C = typename Store<PREC>::C;
    using T = typename Store<PREC>::T;

    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool active = k < a.nfluid;
    const int64_t St = a.S;
    const Coll<C>& cp = coll_of<C>(a);
    Moments<C> mo;
    Pre<C> pr;
    bool used_fb = false;
    if (active) {
        const S* A = (const S*)a.src;
        C h[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const S* p = A + (int64_t)i * St + k;
            h[i] = decode<PREC>(NT ? ld_stream(p) : *p, L::w[i], a.h16_scale);
        }
        C tau_prev = C(0);
        if constexpr (has_tau(OP)) tau_prev = (C)((const T*)a.tau)[k];

        collide_node<LAT, OP, PREC>(h, tau_prev, a.fallback, a.cd, cp, mo, pr, used_fb);

        S* B = (S*)a.dst;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            S* p = B + (int64_t)opp(i) * St + k;
            const S v = encode<PREC>(h[i], L::w[i], a.h16_inv);
            if constexpr (NT) st_stream(v, p);
            else *p = v;
        }
        if constexpr (has_tau(OP)) ((T*)a.tau)[k] = (T)pr.tau_p;
    }
    if constexpr (MON)
        monitor_block<C>(active, mo, pr, cp, used_fb, a.partials + (int64_t)blockIdx.x * MP_COUNT, a.uprev, k, St);
}

// Position of the set bit of v with r set bits below it (r < popcount(v)).
__device__ __forceinline__ int select_bit(uint64_t v, uint32_t r)
{
    int pos = 0;
    uint32_t c = (uint32_t)__popc((uint32_t)v);
    if (r >= c) { r -= c; pos = 32; v >>= 32; }
    c = (uint32_t)__popc((uint32_t)v & 0xFFFFu);
    if (r >= c) { r -= c; pos += 16; v >>= 16; }
    c = (uint32_t)__popc((uint32_t)v & 0xFFu);
    if (r >= c) { r -= c; pos += 8; v >>= 8; }
    c = (uint32_t)__popc((uint32_t)v & 0xFu);
    if (r >= c) { r -= c; pos += 4; v >>= 4; }
    c = (uint32_t)__popc((uint32_t)v & 0x3u);
    if (r >= c) { r -= c; pos += 2; v >>= 2; }
    if (r >= (uint32_t)(v & 1u)) pos += 1;
    return pos;
}

// Compact layout, neighbour phases (AA pull, A/B) with one thread per fluid
// slot: a wavefront is 64 consecutive slots, so every lane is busy and the
// runs start on 64-slot boundaries whatever the solid pattern (the
// row-segment kernel above leaves the lanes of solid nodes idle and cuts the
// runs where the rows' fluid counts fall).  Each lane finds its word by a
// binary search between the words of its group's first slot and of the next
// group's, its x by selecting the bit, and the slots of its 26 neighbours by
// rank in the 9 neighbouring rows; slots of one row are consecutive, so
// x - 1 and x + 1 are the rank -1 / +1 neighbours except across the
// periodic x boundary.  Blocks go to the XCDs as 8 contiguous slot ranges.
template <int LAT, int OP, int PREC, int PAT, bool MON>
__global__ __launch_bounds__(kMaxBlockThreads) void k_pull_slots(const StepArgs a)
{
    using L = Lattice<LAT>;
    constexpr int Q = L::Q;
    constexpr int D = L::D;
    using S = typename Store<PREC>::S;
    using C = typename Store<PREC>::C;
    using T = typename Store<PREC>::T;
    static_assert(PAT == PAT_AB || PAT == PAT_AA_PULL, "neighbour phases only");

    const int64_t nblk = (a.nfluid + 255) >> 8;
    const int b = blockIdx.x;
    const int64_t cb = (int64_t)(b & 7) * a.slot_bpx + (b >> 3);
    if (cb >= nblk) return;  // whole block leaves together
    const int64_t k = cb * 256 + threadIdx.x;
    const bool active = k < a.nfluid;
    const int64_t St = a.S;

    // nbf: fluid flag of x + d, bit (dx+1) + 3 r with r = (dy+1) + 3 (dz+1);
    // im[r]: slot of x in row r (x itself if fluid, else the next fluid
    // node); wr[r]: slot of the periodic image across the x boundary
    // (node nx-1 for x = 0, node 0 for x = nx-1).
    uint32_t nbf = 0;
    uint32_t im[9], wr[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) im[r] = wr[r] = 0;
    int x = 0;
    if (active) {
        uint32_t lo = a.wstart[k >> 6];
        uint32_t hi = ((k >> 6) + 1 < a.ngroups) ? a.wstart[(k >> 6) + 1] : (uint32_t)(a.nwords - 1);
        while (lo < hi) {  // last word whose base is <= k: the one holding slot k
            const uint32_t mid = (lo + hi + 1) >> 1;
            if ((int64_t)a.wbase[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t row = lo / (uint32_t)a.W;
        const int wx = (int)(lo - row * (uint32_t)a.W);
        const int bp = select_bit(a.bits[lo], (uint32_t)(k - (int64_t)a.wbase[lo]));
        x = wx * 64 + bp;
        const int y = (int)(row % (uint32_t)a.ny);
        const int z = (int)(row / (uint32_t)a.ny);
        const uint64_t below = (1ull << bp) - 1ull;
        const int wl = (a.nx - 1) >> 6, bl = (a.nx - 1) & 63;  // last node of a row
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz) {
            if (D == 2 && dz != 0) continue;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                int yy = y + dy, zz = z + dz;
                bool rv = true;
                if (yy < 0 || yy >= a.ny) {
                    if (a.per[1]) yy = (yy + a.ny) % a.ny;
                    else rv = false;
                }
                if (zz < 0 || zz >= a.nz) {
                    if (a.per[2]) zz = (zz + a.nz) % a.nz;
                    else rv = false;
                }
                if (!rv) continue;
                const int r = (dy + 1) + 3 * (dz + 1);
                const int64_t rw = ((int64_t)yy + (int64_t)a.ny * zz) * a.W;
                const uint64_t word = a.bits[rw + wx];
                bool fL = false, fR = false;
                uint32_t wrap = 0;
                if (bp > 0) fL = (word >> (bp - 1)) & 1;
                else if (x > 0) fL = a.bits[rw + wx - 1] >> 63;
                else if (a.per[0]) {
                    const uint64_t lw = a.bits[rw + wl];
                    fL = (lw >> bl) & 1;
                    wrap = a.wbase[rw + wl] + (uint32_t)__popcll(lw & ((1ull << bl) - 1ull));
                }
                if (x + 1 < a.nx) fR = (bp < 63) ? ((word >> (bp + 1)) & 1) : (a.bits[rw + wx + 1] & 1);
                else if (a.per[0]) {
                    fR = a.bits[rw] & 1;
                    if (x > 0) wrap = a.wbase[rw];  // nx = 1: the left image above is this node
                }
                nbf |= (fL ? 1u : 0u) << (3 * r + 0);
                nbf |= (uint32_t)((word >> bp) & 1) << (3 * r + 1);
                nbf |= (fR ? 1u : 0u) << (3 * r + 2);
                im[r] = a.wbase[rw + wx] + (uint32_t)__popcll(word & below);
                wr[r] = wrap;
            }
        }
    }
    // slot of the neighbour x + (dx, row r) (valid when it is fluid)
    auto nbi = [&](int dx, int r) -> uint32_t {
        if (dx == 0) return im[r];
        if (dx < 0) return x > 0 ? im[r] - 1u : wr[r];
        return x + 1 < a.nx ? im[r] + ((nbf >> (3 * r + 1)) & 1u) : wr[r];
    };

    C h[Q];
    C tau_prev = C(0);
    const Coll<C>& cp = coll_of<C>(a);
    Moments<C> mo;
    Pre<C> pr;
    bool used_fb = false;
    if (active) {
        const S* A = (const S*)a.src;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int r = (1 - L::cy[i]) + 3 * (1 - L::cz[i]);  // row of x - c_i
            const bool fl = (nbf >> (3 * r + 1 - L::cx[i])) & 1;
            // branch-free: the 32-bit slot and one of two wave-uniform array bases
            const int dn = PAT == PAT_AB ? i : opp(i), db = PAT == PAT_AB ? opp(i) : i;
            const uint32_t sl = fl ? nbi(-L::cx[i], r) : (uint32_t)k;
            h[i] = decode<PREC>((fl ? A + dn * St : A + db * St)[sl], L::w[i], a.h16_scale);
        }
        if constexpr (has_tau(OP)) tau_prev = (C)((const T*)a.tau)[k];

        collide_node<LAT, OP, PREC>(h, tau_prev, a.fallback, a.cd, cp, mo, pr, used_fb);

        if constexpr (PAT == PAT_AA_PULL) {
            // The store of direction opp(i) goes where the load of i came
            // from; hiding the indices' history from the optimiser keeps it
            // from holding the 27 load addresses through the collision
            // (they cost more registers than rebuilding them).  No
            // instruction is emitted.
#pragma unroll
            for (int r = 0; r < 9; ++r) asm volatile("" : "+v"(im[r]), "+v"(wr[r]));
            asm volatile("" : "+v"(nbf));
        }
        S* B = (S*)a.dst;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            S* p;
            if constexpr (PAT == PAT_AB) {
                p = B + (int64_t)i * St + k;
            } else {
                const int r = (1 + L::cy[i]) + 3 * (1 + L::cz[i]);  // row of x + c_i
                const bool fl = (nbf >> (3 * r + 1 + L::cx[i])) & 1;
                const uint32_t sl = fl ? nbi(L::cx[i], r) : (uint32_t)k;
                p = (fl ? B + i * St : B + opp(i) * St) + sl;
            }
            *p = encode<PREC>(h[i], L::w[i], a.h16_inv);
        }
        if constexpr (has_tau(OP)) ((T*)a.tau)[k] = (T)pr.tau_p;
    }
    if constexpr (MON)
        monitor_block<C>(active, mo, pr, cp, used_fb, a.partials + cb * MP_COUNT, a.uprev, k, St);
}

template <int LAT, int OP, int PREC, int PAT, bool MON>
static hipError_t go_step(int layout, const StepArgs& a, hipStream_t s)
{
    const int threads = a.tx * a.ty * a.tz;
    const dim3 grid(8 * a.tiles_per_xcd);
    if (layout == LAYOUT_COMPACT && PAT == PAT_AA_LOCAL) {
        const int64_t blocks = (a.nfluid + 255) / 256;
        if (blocks > 0) {
            if (a.stream_hint)
                hipLaunchKernelGGL((k_local_slots<LAT, OP, PREC, MON, true>), dim3((unsigned)blocks), dim3(256), 0, s, a);
            else
                hipLaunchKernelGGL((k_local_slots<LAT, OP, PREC, MON, false>), dim3((unsigned)blocks), dim3(256), 0, s, a);
        }
    } else if (layout == LAYOUT_COMPACT && a.pull_slots) {
        if (a.nfluid > 0) {
            if constexpr (PAT != PAT_AA_LOCAL)
                hipLaunchKernelGGL((k_pull_slots<LAT, OP, PREC, PAT, MON>), dim3(8u * (unsigned)a.slot_bpx), dim3(256),
                                   0, s, a);
        }
    } else if (layout == LAYOUT_COMPACT) {
        if constexpr (PAT != PAT_AA_LOCAL) {
            if (a.buf_rows)
                hipLaunchKernelGGL((k_step_rows<LAT, OP, PREC, PAT, MON>), grid, dim3(threads), 0, s, a, a.recs);
            else
                hipLaunchKernelGGL((k_step_compact<LAT, OP, PREC, PAT, MON>), grid, dim3(threads), 0, s, a, a.recs);
        }
    } else {
        const int hz = (Lattice<LAT>::D == 3) ? a.tz + 2 : 1;
        const size_t sh = (PAT != PAT_AA_LOCAL) ? (size_t)(a.tx + 2) * (a.ty + 2) * hz : 0;
        hipLaunchKernelGGL((k_step<LAT, OP, PREC, PAT, MON>), grid, dim3(threads), sh, s, a);
    }
    return hipGetLastError();
}

template <int LAT, int OP, int PREC>
static hipError_t go_pat(int pat, bool mon, int layout, const StepArgs& a, hipStream_t s)
{
    switch (pat) {
    case PAT_AB:
        return mon ? go_step<LAT, OP, PREC, PAT_AB, true>(layout, a, s)
                   : go_step<LAT, OP, PREC, PAT_AB, false>(layout, a, s);
    case PAT_AA_PULL:
        return mon ? go_step<LAT, OP, PREC, PAT_AA_PULL, true>(layout, a, s)
                   : go_step<LAT, OP, PREC, PAT_AA_PULL, false>(layout, a, s);
    case PAT_AA_LOCAL:
        return mon ? go_step<LAT, OP, PREC, PAT_AA_LOCAL, true>(layout, a, s)
                   : go_step<LAT, OP, PREC, PAT_AA_LOCAL, false>(layout, a, s);
    default: return hipErrorInvalidValue;
    }
}

// One lattice and one storage precision per translation unit.  Reduced
// precision adds the OP_FB variants (FP64 redo of near-yield nodes).
template <int LAT, int PREC>
hipError_t launch_step_prec(int op, int pat, bool mon, int layout, const StepArgs& a, hipStream_t s)
{
    constexpr int FB = PREC != PREC_F64 ? OP_FB : 0;
    switch (op) {
    case OP_PR: return go_pat<LAT, OP_PR, PREC>(pat, mon, layout, a, s);
    case OP_PRI: return go_pat<LAT, OP_PRI, PREC>(pat, mon, layout, a, s);
    case OP_PR | OP_MRT: return go_pat<LAT, OP_PR | OP_MRT, PREC>(pat, mon, layout, a, s);
    case OP_PRI | OP_MRT: return go_pat<LAT, OP_PRI | OP_MRT, PREC>(pat, mon, layout, a, s);
    case OP_IR: return go_pat<LAT, OP_IR, PREC>(pat, mon, layout, a, s);
    case OP_IRHB: return go_pat<LAT, OP_IRHB, PREC>(pat, mon, layout, a, s);
    default: break;
    }
    if constexpr (FB != 0) {
        switch (op) {
        case OP_PR | FB: return go_pat<LAT, OP_PR | FB, PREC>(pat, mon, layout, a, s);
        case OP_PRI | FB: return go_pat<LAT, OP_PRI | FB, PREC>(pat, mon, layout, a, s);
        case OP_PR | OP_MRT | FB: return go_pat<LAT, OP_PR | OP_MRT | FB, PREC>(pat, mon, layout, a, s);
        case OP_PRI | OP_MRT | FB: return go_pat<LAT, OP_PRI | OP_MRT | FB, PREC>(pat, mon, layout, a, s);
        case OP_IR | FB: return go_pat<LAT, OP_IR | FB, PREC>(pat, mon, layout, a, s);
        case OP_IRHB | FB: return go_pat<LAT, OP_IRHB | FB, PREC>(pat, mon, layout, a, s);
        default: break;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace lbm
