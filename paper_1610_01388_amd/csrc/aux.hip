// aux.hip -- node-range kernels around the step: initial state, moments
// readout, monitors on demand, population read/write, and the deterministic
// finalisation of monitor partial sums.  None of these is on the hot loop;
// they favour plain 1-D indexing over tiling.
#include <type_traits>

#include "device_common.hpp"

namespace lbm {

// Layout of the stored state (NodeArgs::layout):
//  0: post-collision, natural slots  (A/B; slot i at x holds P_i(x))
//  1: post-collision, swapped slots  (AA after an even number of steps;
//     slot opp(i) at x holds P_i(x))
//  2: streamed, natural slots        (AA after an odd number of steps; slot
//     i at x holds P_i(x - c_i), or P_opp(i)(x) behind a solid / wall)
enum { LAY_POST = 0, LAY_POST_SWAPPED = 1, LAY_STREAMED = 2 };

__device__ __forceinline__ void node_xyz(int64_t n, int nx, int ny, int& x, int& y, int& z)
{
    x = (int)(n % nx);
    const int64_t r = n / nx;
    y = (int)(r % ny);
    z = (int)(r / ny);
}

// Population slot of node (x, y, z) (inside the box), or -1 if it is solid.
__device__ __forceinline__ int64_t slot_of(const NodeArgs& a, int x, int y, int z)
{
    if (a.compact) {
        const int64_t row = ((int64_t)y + (int64_t)a.ny * z) * a.W + (x >> 6);
        const uint64_t word = a.bits[row];
        if (!((word >> (x & 63)) & 1)) return -1;
        return (int64_t)a.wbase[row] + __popcll(word & ((1ull << (x & 63)) - 1ull));
    }
    const int64_t n = x + (int64_t)a.nx * (y + (int64_t)a.ny * z);
    if (!a.mask) return n;  // no interior solids (batched simulations)
    return a.mask[n] ? -1 : n;
}

// Slot of the neighbour at (x,y,z) + c, or -1 when it is solid or lies
// beyond a wall face; periodic axes wrap.
__device__ __forceinline__ int64_t neighbour(const NodeArgs& a, int x, int y, int z, int cx, int cy, int cz)
{
    int p[3] = {x + cx, y + cy, z + cz};
    const int n3[3] = {a.nx, a.ny, a.nz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (p[k] < 0 || p[k] >= n3[k]) {
            if (!a.per[k]) return -1;
            p[k] = (p[k] + n3[k]) % n3[k];
        }
    }
    return slot_of(a, p[0], p[1], p[2]);
}

template <class C> __device__ __forceinline__ const Coll<C>& ncoll(const NodeArgs& a);
template <> __device__ __forceinline__ const Coll<double>& ncoll<double>(const NodeArgs& a) { return a.cd; }
template <> __device__ __forceinline__ const Coll<float>& ncoll<float>(const NodeArgs& a) { return a.cf; }

// Pre-collision populations (deviations) the next step would see at the
// fluid node (x, y, z) with slot k.
template <int LAT, int PREC>
__device__ __forceinline__ void gather(const NodeArgs& a, int64_t k, int x, int y, int z,
                                       typename Store<PREC>::C (&h)[Lattice<LAT>::Q])
{
    using L = Lattice<LAT>;
    using S = typename Store<PREC>::S;
    const S* A = (const S*)a.pdf;
    const int64_t St = a.S;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        int64_t idx;
        if (a.layout == LAY_STREAMED) {
            idx = (int64_t)i * St + k;
        } else {
            const int64_t src = neighbour(a, x, y, z, -L::cx[i], -L::cy[i], -L::cz[i]);
            if (a.layout == LAY_POST)
                idx = src >= 0 ? (int64_t)i * St + src : (int64_t)opp(i) * St + k;
            else
                idx = src >= 0 ? (int64_t)opp(i) * St + src : (int64_t)i * St + k;
        }
        h[i] = decode<PREC>(A[idx], L::w[i], a.h16_scale);
    }
}

// Moments of node n0 + j of the current state: false for a solid node (or j
// past the range), else true with rho, the output velocity uo and the
// rheology state pr.
template <int LAT, int OP, int PREC>
__device__ __forceinline__ bool node_state(const NodeArgs& a, int64_t j, int64_t& k, Pre<typename Store<PREC>::C>& pr,
                                           typename Store<PREC>::C (&uo)[3])
{
    using L = Lattice<LAT>;
    using C = typename Store<PREC>::C;
    using T = typename Store<PREC>::T;
    k = -1;
    if (j >= a.count) return false;
    int x, y, z;
    node_xyz(a.n0 + j, a.nx, a.ny, x, y, z);
    k = slot_of(a, x, y, z);
    if (k < 0) return false;
    const Coll<C>& cp = ncoll<C>(a);
    C h[L::Q];
    gather<LAT, PREC>(a, k, x, y, z, h);
    const C tau_prev = has_tau(OP) ? (C)((const T*)a.tau)[k] : C(0);
    const Moments<C> mo = moments<LAT>(h);
    pr = rheology<LAT, OP>(mo, cp, tau_prev);
    out_velocity(mo, pr, cp, uo);
    return true;
}

// Readout of the current state: per-node moments into staging
// (out[0..count) rho, out[count..4count) u component-major, out[4count..5count)
// nu_app; out_flags unyielded), or (reduce) per-block monitor partials.  The
// reduction walks the nodes with a grid stride, so a grid smaller than one
// block per 256 nodes still covers them all (with one block per 256 nodes,
// every thread takes one node).
template <int LAT, int OP, int PREC>
__global__ __launch_bounds__(kMaxBlockThreads) void k_readout(const NodeArgs a)
{
    using C = typename Store<PREC>::C;
    const int64_t j0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Pre<C> pr;
    C uo[3] = {C(0), C(0), C(0)};
    int64_t k;
    if (a.reduce) {
        double v[MP_COUNT];
#pragma unroll
        for (int q = 0; q < MP_COUNT; ++q) v[q] = 0.0;
        for (int64_t j = j0; j < a.count; j += (int64_t)gridDim.x * blockDim.x) {
            if (!node_state<LAT, OP, PREC>(a, j, k, pr, uo)) continue;
            double w[MP_COUNT];
#pragma unroll
            for (int q = 0; q < MP_COUNT; ++q) w[q] = 0.0;
            const double ux = uo[0], uy = uo[1], uz = uo[2], rho = pr.rho;
            const bool bad = !isfinite(rho) || !isfinite(ux) || !isfinite(uy) || !isfinite(uz);
            w[MP_UX] = ux;
            w[MP_UY] = uy;
            w[MP_UZ] = uz;
            w[MP_MASS] = rho;
            w[MP_UMAX] = bad ? INFINITY : sqrt(ux * ux + uy * uy + uz * uz);
            w[MP_UNYIELDED] = pr.unyielded ? 1.0 : 0.0;
            w[MP_NONFINITE] = bad ? 1.0 : 0.0;
            w[MP_FLUID] = 1.0;
            if (a.uprev) residual_terms(ux, uy, uz, bad, a.uprev + k, a.S, w);
#pragma unroll
            for (int q = 0; q < MP_COUNT; ++q) v[q] = mp_is_max(q) ? fmax(v[q], w[q]) : v[q] + w[q];
        }
        block_reduce_store<MP_COUNT>(v, a.partials + (int64_t)blockIdx.x * MP_COUNT);
        return;
    }
    const bool active = node_state<LAT, OP, PREC>(a, j0, k, pr, uo);
    if (j0 >= a.count) return;
    const int64_t c = a.count;
    a.out[j0] = active ? (double)pr.rho : 0.0;
    a.out[c + j0] = active ? (double)uo[0] : 0.0;
    a.out[2 * c + j0] = active ? (double)uo[1] : 0.0;
    a.out[3 * c + j0] = active ? (double)uo[2] : 0.0;
    a.out[4 * c + j0] = active ? (double)pr.nu_app : 0.0;
    a.out_flags[j0] = active ? (uint8_t)pr.unyielded : (uint8_t)0;
}

// Equilibrium f_eq(rho, u0) (Sec. 2.1, Eq. 12) as the post-collision state;
// stored as deviations from w rho0, in the layout given (0 or 1).  Dense
// storage also clears the slots of solid nodes.
template <int LAT, int OP, int PREC>
__global__ __launch_bounds__(kMaxBlockThreads) void k_init(const NodeArgs a, double rho)
{
    using L = Lattice<LAT>;
    using S = typename Store<PREC>::S;
    using T = typename Store<PREC>::T;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
    int x, y, z;
    node_xyz(n, a.nx, a.ny, x, y, z);
    int64_t k = slot_of(a, x, y, z);
    const bool solid = k < 0;
    if (solid) {
        if (a.compact) return;
        k = n;
    }
    S* A = (S*)a.pdf;
    const double u0[3] = {a.u0[0], a.u0[1], a.u0[2]};
    const double uu = u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double cu = L::cx[i] * u0[0] + L::cy[i] * u0[1] + L::cz[i] * u0[2];
        const double feq = rho * L::w[i] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        const double hdev = solid ? 0.0 : feq - L::w[i] * a.cd.rho0;
        const int slot = (a.layout == LAY_POST_SWAPPED) ? opp(i) : i;
        A[(int64_t)slot * a.S + k] = encode<PREC>((typename Store<PREC>::C)hdev, L::w[i], a.h16_inv);
    }
    if (has_tau(OP) && a.tau) {
        const double nu0 = a.cd.nu_p + a.cd.m * a.cd.sigma_y / rho;
        ((T*)a.tau)[k] = (T)(0.5 + 3.0 * nu0);
    }
}

// Write full populations P (staging: q blocks of count doubles, node order)
// and tau into storage in layout 0 or 1.  Solid nodes carry no state.
template <int LAT, int PREC>
__global__ __launch_bounds__(kMaxBlockThreads) void k_pop_write(const NodeArgs a)
{
    using L = Lattice<LAT>;
    using S = typename Store<PREC>::S;
    using T = typename Store<PREC>::T;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.count) return;
    const int64_t n = a.n0 + j;
    int x, y, z;
    node_xyz(n, a.nx, a.ny, x, y, z);
    const int64_t k = slot_of(a, x, y, z);
    if (k < 0) return;
    S* A = (S*)a.pdf;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double hdev = a.out[(int64_t)i * a.count + j] - L::w[i] * a.cd.rho0;
        const int slot = (a.layout == LAY_POST_SWAPPED) ? opp(i) : i;
        A[(int64_t)slot * a.S + k] = encode<PREC>((typename Store<PREC>::C)hdev, L::w[i], a.h16_inv);
    }
    if (a.tau) ((T*)a.tau)[k] = (T)a.out[(int64_t)L::Q * a.count + j];
}

// Read the post-collision populations P of the last step (full f) and tau
// in node order (solid nodes report 0).  Layout 2 undoes the push of the
// last AA step: P_i(x) sits in slot i of x + c_i, or in slot opp(i) of x when
// x + c_i is solid or beyond a wall.
template <int LAT, int PREC>
__global__ __launch_bounds__(kMaxBlockThreads) void k_pop_read(const NodeArgs a)
{
    using L = Lattice<LAT>;
    using S = typename Store<PREC>::S;
    using T = typename Store<PREC>::T;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.count) return;
    const int64_t n = a.n0 + j;
    const S* A = (const S*)a.pdf;
    int x, y, z;
    node_xyz(n, a.nx, a.ny, x, y, z);
    const int64_t k = slot_of(a, x, y, z);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        double v = 0.0;
        if (k >= 0) {
            int64_t idx;
            if (a.layout == LAY_POST) {
                idx = (int64_t)i * a.S + k;
            } else if (a.layout == LAY_POST_SWAPPED) {
                idx = (int64_t)opp(i) * a.S + k;
            } else {
                const int64_t dst = neighbour(a, x, y, z, L::cx[i], L::cy[i], L::cz[i]);
                idx = dst >= 0 ? (int64_t)i * a.S + dst : (int64_t)opp(i) * a.S + k;
            }
            v = (double)decode<PREC>(A[idx], L::w[i], a.h16_scale) + L::w[i] * a.cd.rho0;
        }
        a.out[(int64_t)i * a.count + j] = v;
    }
    if (a.tau) a.out[(int64_t)L::Q * a.count + j] = k >= 0 ? (double)((const T*)a.tau)[k] : 0.0;
}

// Sum per-block partials in a fixed order into one lbm_monitor record.
struct MonitorRecord {
    int64_t step;
    double flux[3];
    double mass;
    double umax;
    int64_t fluid_nodes, unyielded, fallback_nodes, nonfinite;
    double residual, du_max;
};

__device__ __forceinline__ void fill_record(MonitorRecord* rec, const double (&r)[MP_COUNT], double ntotal)
{
    rec->flux[0] = r[MP_UX] / ntotal;
    rec->flux[1] = r[MP_UY] / ntotal;
    rec->flux[2] = r[MP_UZ] / ntotal;
    rec->mass = r[MP_MASS];
    rec->umax = r[MP_UMAX];
    rec->fluid_nodes = (int64_t)r[MP_FLUID];
    rec->unyielded = (int64_t)r[MP_UNYIELDED];
    rec->fallback_nodes = (int64_t)r[MP_FALLBACK];
    rec->nonfinite = (int64_t)r[MP_NONFINITE];
    rec->residual = r[MP_U2] > 0.0 ? r[MP_DU2] / r[MP_U2] : 0.0;
    rec->du_max = r[MP_DUMAX];
}

__global__ __launch_bounds__(kMaxBlockThreads) void k_finalize(const double* parts, int64_t np, MonitorRecord* rec,
                                                  int64_t step, double ntotal)
{
    __shared__ double red[256][MP_COUNT];
    double v[MP_COUNT];
#pragma unroll
    for (int k = 0; k < MP_COUNT; ++k) v[k] = 0.0;
    for (int64_t j = threadIdx.x; j < np; j += 256) {
#pragma unroll
        for (int k = 0; k < MP_COUNT; ++k) {
            const double o = parts[j * MP_COUNT + k];
            v[k] = mp_is_max(k) ? fmax(v[k], o) : v[k] + o;
        }
    }
#pragma unroll
    for (int k = 0; k < MP_COUNT; ++k) red[threadIdx.x][k] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < MP_COUNT; ++k)
                red[threadIdx.x][k] = mp_is_max(k) ? fmax(red[threadIdx.x][k], red[threadIdx.x + s][k])
                                                     : red[threadIdx.x][k] + red[threadIdx.x + s][k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        rec->step = step;
        fill_record(rec, red[0], ntotal);
    }
}

// Fused monitors of a domain: the same reduction, into ring slot
// (*counter mod capacity), then the counter advances (one block, so the
// read and the increment need no atomics).  The ring position comes from the
// device, so a captured graph replayed several times fills consecutive slots.
__global__ __launch_bounds__(kMaxBlockThreads) void k_finalize_ring(const double* parts, int64_t np, MonitorRecord* ring,
                                                       int64_t* counter, int capacity, int64_t step, double ntotal)
{
    __shared__ double red[256][MP_COUNT];
    double v[MP_COUNT];
#pragma unroll
    for (int k = 0; k < MP_COUNT; ++k) v[k] = 0.0;
    for (int64_t j = threadIdx.x; j < np; j += 256) {
#pragma unroll
        for (int k = 0; k < MP_COUNT; ++k) {
            const double o = parts[j * MP_COUNT + k];
            v[k] = mp_is_max(k) ? fmax(v[k], o) : v[k] + o;
        }
    }
#pragma unroll
    for (int k = 0; k < MP_COUNT; ++k) red[threadIdx.x][k] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < MP_COUNT; ++k)
                red[threadIdx.x][k] = mp_is_max(k) ? fmax(red[threadIdx.x][k], red[threadIdx.x + s][k])
                                                     : red[threadIdx.x][k] + red[threadIdx.x + s][k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t c = *counter;
        MonitorRecord* rec = ring + (c % capacity);
        rec->step = step;
        fill_record(rec, red[0], ntotal);
        *counter = c + 1;
    }
}

// Batched monitors: one block per simulation sums its work items' partials
// in a fixed order into record[(counter mod capacity) * nsims + sim].
__global__ __launch_bounds__(kMaxBlockThreads) void k_batch_finalize(const double* parts, const BatchSim* sims, int nsims,
                                                        MonitorRecord* records, const int64_t* counter,
                                                        int64_t step, int capacity)
{
    __shared__ double red[256][MP_COUNT];
    const int sim = blockIdx.x;
    const BatchSim& sm = sims[sim];
    double v[MP_COUNT];
#pragma unroll
    for (int k = 0; k < MP_COUNT; ++k) v[k] = 0.0;
    for (int j = threadIdx.x; j < sm.nitems; j += 256) {
        const double* p = parts + (int64_t)(sm.item0 + j) * MP_COUNT;
#pragma unroll
        for (int k = 0; k < MP_COUNT; ++k) v[k] = mp_is_max(k) ? fmax(v[k], p[k]) : v[k] + p[k];
    }
#pragma unroll
    for (int k = 0; k < MP_COUNT; ++k) red[threadIdx.x][k] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < MP_COUNT; ++k)
                red[threadIdx.x][k] = mp_is_max(k) ? fmax(red[threadIdx.x][k], red[threadIdx.x + s][k])
                                                     : red[threadIdx.x][k] + red[threadIdx.x + s][k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t c = *counter;
        MonitorRecord* rec = records + (c % capacity) * nsims + sim;
        const double ntotal = (double)sm.N;
        rec->step = c;  // record number; the host maps it to the time step
        fill_record(rec, red[0], ntotal);
    }
}

__global__ void k_batch_tick(int64_t* counter)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter += 1;
}

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int V> using ic = std::integral_constant<int, V>;

// Call f(ic<LAT>, ic<PREC>) for runtime lattice and precision.
template <class F>
static hipError_t dispatch_lat_prec(int lat, int prec, F&& f)
{
    switch (lat * 3 + prec) {
    case 0: return f(ic<0>{}, ic<0>{});
    case 1: return f(ic<0>{}, ic<1>{});
    case 2: return f(ic<0>{}, ic<2>{});
    case 3: return f(ic<1>{}, ic<0>{});
    case 4: return f(ic<1>{}, ic<1>{});
    case 5: return f(ic<1>{}, ic<2>{});
    case 6: return f(ic<2>{}, ic<0>{});
    case 7: return f(ic<2>{}, ic<1>{});
    case 8: return f(ic<2>{}, ic<2>{});
    default: return hipErrorInvalidValue;
    }
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_readout(int lat, int op, int prec, const NodeArgs& a, hipStream_t s, int64_t* nblocks,
                          int64_t max_blocks)
{
    int64_t nb = (int64_t)nblk(a.count);
    if (a.reduce && max_blocks > 0 && nb > max_blocks) nb = max_blocks;  // grid-stride reduction
    if (nblocks) *nblocks = nb;
    if (a.count == 0) return hipSuccess;
    const dim3 grid((unsigned)nb);
    return dispatch_lat_prec(lat, prec, [&](auto L, auto P) {
        if (op == OP_PR)
            hipLaunchKernelGGL((k_readout<decltype(L)::value, OP_PR, decltype(P)::value>), grid, dim3(256), 0, s, a);
        else if (op == OP_PRI)
            hipLaunchKernelGGL((k_readout<decltype(L)::value, OP_PRI, decltype(P)::value>), grid, dim3(256), 0, s, a);
        else if (op == (OP_PR | OP_MRT))
            hipLaunchKernelGGL((k_readout<decltype(L)::value, OP_PR | OP_MRT, decltype(P)::value>), grid, dim3(256), 0,
                               s, a);
        else if (op == (OP_PRI | OP_MRT))
            hipLaunchKernelGGL((k_readout<decltype(L)::value, OP_PRI | OP_MRT, decltype(P)::value>), grid, dim3(256),
                               0, s, a);
        else  // IR and IRHB: the readout (velocity, yield flag) does not depend on the law's solve
            hipLaunchKernelGGL((k_readout<decltype(L)::value, OP_IR, decltype(P)::value>), grid, dim3(256), 0, s, a);
        return hipGetLastError();
    });
}

hipError_t launch_init(int lat, int op, int prec, const NodeArgs& a, double rho, hipStream_t s)
{
    op = op_base(op);  // the initial state does not depend on the base collision
    return dispatch_lat_prec(lat, prec, [&](auto L, auto P) {
        if (op == OP_PR)
            hipLaunchKernelGGL((k_init<decltype(L)::value, OP_PR, decltype(P)::value>), dim3(nblk(a.N)), dim3(256),
                               0, s, a, rho);
        else if (op == OP_PRI)
            hipLaunchKernelGGL((k_init<decltype(L)::value, OP_PRI, decltype(P)::value>), dim3(nblk(a.N)), dim3(256),
                               0, s, a, rho);
        else
            hipLaunchKernelGGL((k_init<decltype(L)::value, OP_IR, decltype(P)::value>), dim3(nblk(a.N)), dim3(256),
                               0, s, a, rho);
        return hipGetLastError();
    });
}

hipError_t launch_pop_write(int lat, int prec, const NodeArgs& a, hipStream_t s)
{
    if (a.count == 0) return hipSuccess;
    return dispatch_lat_prec(lat, prec, [&](auto L, auto P) {
        hipLaunchKernelGGL((k_pop_write<decltype(L)::value, decltype(P)::value>), dim3(nblk(a.count)), dim3(256), 0,
                           s, a);
        return hipGetLastError();
    });
}

hipError_t launch_pop_read(int lat, int prec, const NodeArgs& a, hipStream_t s)
{
    if (a.count == 0) return hipSuccess;
    return dispatch_lat_prec(lat, prec, [&](auto L, auto P) {
        hipLaunchKernelGGL((k_pop_read<decltype(L)::value, decltype(P)::value>), dim3(nblk(a.count)), dim3(256), 0,
                           s, a);
        return hipGetLastError();
    });
}

hipError_t launch_finalize(const double* partials, int64_t nparts, void* record, int64_t step, double ntotal,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, partials, nparts, (MonitorRecord*)record, step, ntotal);
    return hipGetLastError();
}

hipError_t launch_finalize_ring(const double* partials, int64_t nparts, void* ring, int64_t* counter, int capacity,
                                int64_t step, double ntotal, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_ring, dim3(1), dim3(256), 0, s, partials, nparts, (MonitorRecord*)ring, counter,
                       capacity, step, ntotal);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u8, dim3(nblk(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_batch_step(int lat, int prec, int pat, bool mon, const BatchArgs& a, int grid, hipStream_t s)
{
    switch (lat) {
    case 0: return launch_batch_lattice<0>(prec, pat, mon, a, grid, s);
    case 1: return launch_batch_lattice<1>(prec, pat, mon, a, grid, s);
    case 2: return launch_batch_lattice<2>(prec, pat, mon, a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_finalize(const BatchArgs& a, const int* /*unused*/, void* records, const int64_t* counter,
                                 int64_t step, int capacity, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_finalize, dim3(a.nsims), dim3(256), 0, s, a.partials, a.sims, a.nsims,
                       (MonitorRecord*)records, counter, step, capacity);
    return hipGetLastError();
}

hipError_t launch_batch_tick(int64_t* counter, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_tick, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_step(int lat, int op, int prec, int pat, bool mon, int layout, const StepArgs& a, hipStream_t s)
{
    if (lat < 0 || lat > 2 || prec < 0 || prec > 2) return hipErrorInvalidValue;
    static hipError_t (*const table[3][3])(int, int, bool, int, const StepArgs&, hipStream_t) = {
        {launch_step_prec<0, PREC_F64>, launch_step_prec<0, PREC_F32>, launch_step_prec<0, PREC_F16>},
        {launch_step_prec<1, PREC_F64>, launch_step_prec<1, PREC_F32>, launch_step_prec<1, PREC_F16>},
        {launch_step_prec<2, PREC_F64>, launch_step_prec<2, PREC_F32>, launch_step_prec<2, PREC_F16>}};
    return table[lat][prec](op, pat, mon, layout, a, s);
}

}  // namespace lbm
