// device_common.hpp -- storage codec and small device helpers shared by the
// step kernel and the node-range kernels (internal).
#pragma once

#include "kernels.hpp"

namespace lbm {

template <int PREC> struct Store;
template <> struct Store<PREC_F64> { using S = double; using C = double; using T = double; };
template <> struct Store<PREC_F32> { using S = float; using C = float; using T = float; };
template <> struct Store<PREC_F16> { using S = _Float16; using C = float; using T = float; };

template <class C> __device__ __forceinline__ const Coll<C>& coll_of(const StepArgs& a);
template <> __device__ __forceinline__ const Coll<double>& coll_of<double>(const StepArgs& a) { return a.cd; }
template <> __device__ __forceinline__ const Coll<float>& coll_of<float>(const StepArgs& a) { return a.cf; }

// Storage codec.  FP64/FP32 hold h = f - w rho0 directly; FP16 holds
// h * 2^k / w (round to nearest even), decoded to float.
template <int PREC>
__device__ __forceinline__ typename Store<PREC>::C decode(typename Store<PREC>::S v, double w, float scale)
{
    if constexpr (PREC == PREC_F16) return (float)v * ((float)w * scale);
    else return v;
}

template <int PREC>
__device__ __forceinline__ typename Store<PREC>::S encode(typename Store<PREC>::C h, double w, float inv)
{
    if constexpr (PREC == PREC_F16) return (_Float16)(h * ((float)(1.0 / w) * inv));
    else return h;
}

// Streaming access to population storage.  Each element is read once and
// written once per step; with the non-temporal hint on both the loads and
// the stores, the in-place many-array pattern runs about 5% faster on
// gfx950 (hint on one side only: no gain).
template <class S>
__device__ __forceinline__ S ld_stream(const S* p)
{
    return __builtin_nontemporal_load(p);
}
template <class S>
__device__ __forceinline__ void st_stream(S v, S* p)
{
    __builtin_nontemporal_store(v, p);
}

// Wrap a halo coordinate g in [-1, n]: periodic axes wrap, walls give
// "outside" (treated as solid: halfway bounce-back at the face).
__device__ __forceinline__ int wrap_halo(int g, int n, int per, bool& out)
{
    if (g < 0) {
        if (per) return g + n;
        out = true;
        return 0;
    }
    if (g >= n) {
        if (per && g == n) return 0;
        out = true;
        return 0;
    }
    return g;
}

// Residual terms of one node: |u - u_prev|^2, |u|^2 and |u - u_prev|, with
// u_prev the velocity stored at the previous fused monitor (three entries
// `stride` apart).
__device__ __forceinline__ void residual_terms(double ux, double uy, double uz, bool bad, const double* up,
                                               int64_t stride, double (&v)[MP_COUNT])
{
    const double d0 = ux - up[0], d1 = uy - up[stride], d2 = uz - up[2 * stride];
    const double du2 = d0 * d0 + d1 * d1 + d2 * d2;
    v[MP_DU2] = du2;
    v[MP_U2] = ux * ux + uy * uy + uz * uz;
    v[MP_DUMAX] = bad ? INFINITY : sqrt(du2);
}

// Sum (max for the max-type entries) of v over the block into dst.  One
// slot of the shared buffer per wavefront: blocks of at most
// kMaxBlockThreads threads, which every kernel's launch bounds state.
template <int N>
__device__ __forceinline__ void block_reduce_store(double (&v)[N], double* dst)
{
    static_assert(kMaxBlockThreads % 64 == 0, "whole wavefronts per block");
    __shared__ double red[kMaxBlockThreads / 64][N];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double o = __shfl_xor(v[k], off, 64);
            v[k] = mp_is_max(k) ? fmax(v[k], o) : v[k] + o;
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) red[wave][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < N; ++k) {
            double s = red[0][k];
            for (int w = 1; w < nw; ++w) s = mp_is_max(k) ? fmax(s, red[w][k]) : s + red[w][k];
            dst[k] = s;
        }
    }
}

}  // namespace lbm
