// capi.hip -- host side of the C ABI declared in include/lbm.h: validation,
// buffer binding, the step loop (A/B copy swap or AA phase alternation),
// fused monitors, chunked host I/O through a staging area, checkpoints and
// the tile autotuner.  The library never allocates device memory: every
// device buffer is bound by the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host.hpp"
#include "kernels.hpp"
#include "lbm.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(LBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

constexpr int kHistory = 4096;
constexpr size_t kStageMax = size_t(64) << 20;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct MonitorRecord {
    int64_t step;
    double flux[3];
    double mass;
    double umax;
    int64_t fluid_nodes, unyielded, fallback_nodes, nonfinite;
    double residual, du_max;
};
static_assert(sizeof(MonitorRecord) == sizeof(lbm_monitor), "record layout must match lbm_monitor");
static_assert((int)LAYOUT_COMPACT == (int)LBM_COMPACT && (int)LAYOUT_DENSE == (int)LBM_DENSE,
              "kernel layout codes must equal the C ABI's lbm_layout values");
static_assert((int)PREC_F64 == (int)LBM_FP64 && (int)PREC_F32 == (int)LBM_FP32 && (int)PREC_F16 == (int)LBM_FP16,
              "kernel precision codes must equal the C ABI's lbm_precision values");
static_assert((int)OP_PR == (int)LBM_PR && (int)OP_IR == (int)LBM_IR && (int)OP_PRI == (int)LBM_PRI &&
                  (int)OP_IRHB == (int)LBM_IRHB,
              "kernel operator codes must equal the C ABI's lbm_operator values");

// Population arrays carry kStridePad elements of slack beyond the node count
// rounded to 64, room for compact_stride's padding (below 64 KiB per array).
constexpr int64_t kStridePad = 32768;

struct Layout {
    size_t pdf_copy, pdf, tau, mask, part, hist, rec, counter, uprev, stage, work;
    size_t bits_off, base_off, wstart_off, recs_off, mask_compact;  // compact mask: bitmap, word bases, group
                                                                    // words, segment records
    int64_t max_parts, npad;
    int W;
};

int check_desc(const lbm_desc* d)
{
    std::string err;
    const int rc = validate_desc(d, err);
    return rc ? fail(rc, "%s", err.c_str()) : LBM_OK;
}

int check_rheology(const lbm_rheology* r)
{
    std::string err;
    const int rc = validate_rheology(r, err);
    return rc ? fail(rc, "%s", err.c_str()) : LBM_OK;
}

Layout layout_of(const lbm_desc* d, const lbm_rheology* r)
{
    Layout L{};
    const int64_t N = (int64_t)d->nx * d->ny * d->nz;
    const int Q = lattice_q(d->lattice);
    L.npad = (N + 63) / 64 * 64 + kStridePad;
    L.pdf_copy = align_up((size_t)Q * L.npad * prec_bytes(d->precision));
    L.pdf = L.pdf_copy * (d->scheme == LBM_AB ? 2 : 1);
    L.tau = (r && r->op == LBM_PR) ? align_up((size_t)L.npad * (d->precision == LBM_FP64 ? 8 : 4)) : 0;
    L.W = (d->nx + 63) / 64;
    const size_t words = (size_t)L.W * d->ny * d->nz;
    L.bits_off = 0;
    L.base_off = align_up(words * 8);
    L.wstart_off = L.base_off + align_up(words * 4);
    L.recs_off = L.wstart_off + align_up(((size_t)N / 64 + 1) * 4);
    L.mask_compact = L.recs_off + align_up((size_t)L.W * (d->ny + 2) * (d->nz + 2) * sizeof(SegRec));
    L.mask = std::max(align_up((size_t)N), L.mask_compact);
    L.max_parts = N / 32 + 64;
    L.part = 0;
    L.hist = align_up((size_t)L.max_parts * MP_COUNT * sizeof(double));
    L.rec = L.hist + align_up(kHistory * sizeof(MonitorRecord));
    L.counter = L.rec + align_up(sizeof(MonitorRecord));
    L.uprev = L.counter + kAlign;
    L.stage = L.uprev + align_up((size_t)3 * L.npad * sizeof(double));
    size_t stage = std::min(kStageMax, align_up((size_t)N * (Q + 1) * 8));
    stage = std::max(stage, align_up((size_t)(Q + 1) * 8 * 256));
    L.work = L.stage + stage;
    return L;
}

}  // namespace

struct lbm_domain {
    lbm_desc d;
    lbm_rheology r;
    int Q = 0, D = 0;
    int64_t N = 0;
    Layout L{};
    bool bound = false;
    char* pdf = nullptr;
    void* tau = nullptr;
    uint8_t* mask = nullptr;
    char* work = nullptr;
    hipStream_t stream = nullptr;
    int cur = 0;     // A/B: copy holding the current post-collision state
    int parity = 0;  // AA: 0 = post-collision swapped, 1 = streamed natural
    int64_t t = 0;
    int tx = 64, ty = 4, tz = 1;
    int bry = 0, brz = 0;  // tile-order bricks (0 = default for the tile shape)
    int pull_form = LBM_PULL_AUTO;  // compact neighbour phases: slot or row-segment kernel
    int mon_k = 0;
    int64_t hist_written = 0, hist_read = 0;
    std::vector<int64_t> hist_time = std::vector<int64_t>(kHistory, 0);  // time of each ring slot's record
    double umax_limit = 0.1;
    int64_t S = 0;   // direction stride of the population arrays
    int64_t Nf = 0;  // fluid nodes
    // captured-graph stepping: replays of graph_steps launches (0 = eager)
    int graph_steps = 0;
    hipGraphExec_t graph = nullptr;
    hipStream_t cap = nullptr;
    uint64_t gen = 0;        // bumped by every change to what the step launches bake in
    uint64_t graph_gen = 0;  // gen the graph was captured at
    double* scratch = nullptr;  // this GPU's allocation-free monitor scratch (resolved by lbm_bind)
};

namespace {

int ntiles_of(const lbm_domain* dm, int tx, int ty, int tz)
{
    const int64_t nt = (int64_t)((dm->d.nx + tx - 1) / tx) * ((dm->d.ny + ty - 1) / ty) * ((dm->d.nz + tz - 1) / tz);
    return nt > INT32_MAX ? INT32_MAX : (int)nt;
}

int check_tile(const lbm_domain* dm, int tx, int ty, int tz)
{
    static_assert(kMaxBlockThreads == 256, "tile shapes are validated against 256-thread blocks");
    const int th = tx * ty * tz;
    if (tx < 1 || ty < 1 || tz < 1 || (th != 64 && th != 128 && th != 192 && th != 256))
        return fail(LBM_EINVAL, "tile %dx%dx%d: threads must be 64, 128, 192 or 256", tx, ty, tz);
    if (dm->D == 2 && tz != 1) return fail(LBM_EINVAL, "tz must be 1 for D2Q9");
    if (dm->d.layout == LBM_COMPACT && tx != 64 && tx != 128 && tx != 256)
        return fail(LBM_EINVAL, "the compact layout needs tx = 64, 128 or 256 (whole 64-node row segments)");
    if (ntiles_of(dm, tx, ty, tz) > dm->L.max_parts)
        return fail(LBM_EINVAL, "tile %dx%dx%d leaves too many mostly empty tiles for this domain", tx, ty, tz);
    return LBM_OK;
}

// Neighbour-phase kernel in effect for the compact layout: the slot kernel
// keeps every lane busy, the row-segment kernel reads the bitmap through the
// scalar cache but idles the lanes of solid nodes; measured on D3Q27 FP64
// 256^3 boxes, the row kernel leads from 70% fluid up and the slot kernel
// below 40% (1.7x at 15%).
bool pull_slots(const lbm_domain* dm)
{
    if (dm->d.layout != LBM_COMPACT) return false;
    if (dm->pull_form == LBM_PULL_AUTO) return (double)dm->Nf < 0.45 * (double)dm->N;
    return dm->pull_form == LBM_PULL_SLOTS;
}

int pow2ceil(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

void default_tile(lbm_domain* dm)
{
    if (dm->d.layout == LBM_COMPACT) {
        // up to 4 adjacent 64-node segments of one row per block (their shared
        // cache lines then meet in L2; 256x1x1 measured 1.5% faster than
        // 64x4x1 on the 256^3 pack), the largest count that divides the row's
        // segments so that no wavefront sits past the row end (384 wide: 2),
        // the other waves over y, z
        const int sx = dm->L.W % 4 == 0 ? 4 : dm->L.W % 2 == 0 ? 2 : 1;
        dm->tx = 64 * sx;
        dm->ty = std::min(pow2ceil(dm->d.ny), 4 / sx);
        dm->tz = dm->D == 3 ? std::min(pow2ceil(dm->d.nz), 4 / (sx * dm->ty)) : 1;
        return;
    }
    int tx = std::min(pow2ceil(dm->d.nx), 64);
    int ty = std::min(pow2ceil(dm->d.ny), 256 / tx);
    int tz = dm->D == 3 ? std::min(pow2ceil(dm->d.nz), 256 / (tx * ty)) : 1;
    while (tx * ty * tz < 64) {
        if (tx < 64) tx *= 2;
        else ty *= 2;
    }
    dm->tx = tx;
    dm->ty = ty;
    dm->tz = tz;
}

template <class C>
Coll<C> make_coll(const lbm_rheology& r)
{
    Coll<C> c{};
    c.rho0 = (C)r.rho0;
    c.nu_p = (C)r.nu_p;
    c.sigma_y = (C)r.sigma_y;
    c.m = (C)r.m;
    c.gamma_c = (C)(r.gamma_c > 0 ? r.gamma_c : 1e-8);
    c.lambda = (C)r.lambda_trt;
    for (int a = 0; a < 3; ++a) c.g[a] = (C)r.g[a];
    c.sqrt2_sy = (C)(std::sqrt(2.0) * r.sigma_y);
    c.ir_a = (C)((6.0 * r.nu_p - 1.0) / (1.0 + 6.0 * r.nu_p));
    c.ir_b = (C)(2.0 * std::sqrt(2.0) * r.sigma_y / (1.0 + 6.0 * r.nu_p));
    const double gc = r.gamma_c > 0 ? r.gamma_c : 1e-8;
    c.pr_ec = (C)(-std::expm1(-r.m * gc) / gc);
    c.band = (C)r.fallback_band;
    c.axis = r.flow_axis;
    c.mrt_b = (C)r.mrt_bulk;
    c.mrt_e = (C)r.mrt_even;
    c.hb_n = (C)r.hb_n;
    c.hb_c = (C)(3.0 * r.nu_p * std::pow(3.0 / std::sqrt(2.0), r.hb_n - 1.0));
    return c;
}

// Kernel operator code: the ABI operator plus the MRT flag.
int kernel_op(const lbm_rheology& r)
{
    return r.op | ((r.mrt_bulk > 0 || r.mrt_even > 0) ? (int)OP_MRT : 0);
}

char* copy_ptr(lbm_domain* dm, int k) { return dm->pdf + (size_t)k * dm->L.pdf_copy; }

// Layout code of the stored state (see aux.hip).
int state_layout(const lbm_domain* dm)
{
    if (dm->d.scheme == LBM_AB) return 0;
    return dm->parity == 0 ? 1 : 2;
}

NodeArgs node_args(lbm_domain* dm)
{
    NodeArgs a{};
    a.pdf = dm->d.scheme == LBM_AB ? copy_ptr(dm, dm->cur) : dm->pdf;
    a.tau = dm->tau;
    a.mask = dm->mask;
    a.partials = (double*)dm->work;
    a.uprev = (const double*)(dm->work + dm->L.uprev);
    a.N = dm->N;
    a.nx = dm->d.nx;
    a.ny = dm->d.ny;
    a.nz = dm->d.nz;
    for (int k = 0; k < 3; ++k) a.per[k] = dm->d.periodic[k] ? 1 : 0;
    if (dm->D == 2) a.per[2] = 1;
    a.layout = state_layout(dm);
    a.compact = dm->d.layout == LBM_COMPACT ? 1 : 0;
    a.bits = (const uint64_t*)(dm->mask + dm->L.bits_off);
    a.wbase = (const uint32_t*)(dm->mask + dm->L.base_off);
    a.W = dm->L.W;
    a.S = dm->S;
    a.h16_scale = std::ldexp(1.0f, -dm->r.fp16_scale_log2);
    a.h16_inv = std::ldexp(1.0f, dm->r.fp16_scale_log2);
    a.cd = make_coll<double>(dm->r);
    a.cf = make_coll<float>(dm->r);
    return a;
}

// Tile-order bricks: whole rows x bry row-blocks x brz planes.  Default for
// the compact layout: a brick holds about 16 tiles per plane (so
// z-neighbours are ~16 tiles apart in the order) and one slab of planes per
// XCD; the dense layout walks x, y, z plainly (measured faster there).
void tile_order(const lbm_domain* dm, int ntx, int nty, int ntz, int& bry, int& brz)
{
    const bool dense = dm->d.layout == LBM_DENSE;  // the dense kernel keeps the plain order by default
    bry = dm->bry > 0 ? dm->bry : dense ? nty : std::max(1, 16 / std::max(1, ntx));
    brz = dm->brz > 0 ? dm->brz : dense ? ntz : (ntz + 7) / 8;
    bry = std::max(1, std::min(bry, nty));
    brz = std::max(1, std::min(brz, ntz));
}

StepArgs step_args(lbm_domain* dm)
{
    StepArgs a{};
    a.tau = dm->tau;
    a.mask = dm->mask;
    a.bits = (const uint64_t*)(dm->mask + dm->L.bits_off);
    a.wbase = (const uint32_t*)(dm->mask + dm->L.base_off);
    a.wstart = (const uint32_t*)(dm->mask + dm->L.wstart_off);
    a.recs = (const SegRec*)(dm->mask + dm->L.recs_off);
    a.W = dm->L.W;
    a.S = dm->S;
    a.nfluid = dm->Nf;
    a.ngroups = (dm->Nf + 63) / 64;
    a.nwords = (int64_t)dm->L.W * dm->d.ny * dm->d.nz;
    a.slot_bpx = (int)(((dm->Nf + 255) / 256 + 7) / 8);
    a.pull_slots = pull_slots(dm) ? 1 : 0;
    a.buf_rows = 2.0 * (double)dm->S * (double)prec_bytes(dm->d.precision) < 4294967296.0 ? 1 : 0;
    a.partials = (double*)dm->work;
    a.uprev = (double*)(dm->work + dm->L.uprev);
    a.N = dm->N;
    a.nx = dm->d.nx;
    a.ny = dm->d.ny;
    a.nz = dm->d.nz;
    for (int k = 0; k < 3; ++k) a.per[k] = dm->d.periodic[k] ? 1 : 0;
    if (dm->D == 2) a.per[2] = 1;
    a.tx = dm->tx;
    a.ty = dm->ty;
    a.tz = dm->tz;
    a.ntx = (dm->d.nx + dm->tx - 1) / dm->tx;
    a.nty = (dm->d.ny + dm->ty - 1) / dm->ty;
    a.ntz = (dm->d.nz + dm->tz - 1) / dm->tz;
    a.ntiles = a.ntx * a.nty * a.ntz;
    a.tiles_per_xcd = (a.ntiles + 7) / 8;
    tile_order(dm, a.ntx, a.nty, a.ntz, a.bry, a.brz);
    // non-temporal hints when the population state exceeds 512 MiB, twice
    // the 256 MB last-level cache: a state that still partly fits keeps its
    // cache hits
    a.stream_hint = (double)dm->Q * (double)dm->S * (double)prec_bytes(dm->d.precision) > 512.0 * (1 << 20) ? 1 : 0;
    a.fallback = (dm->d.precision != LBM_FP64 && dm->r.fp64_fallback) ? 1 : 0;
    a.h16_scale = std::ldexp(1.0f, -dm->r.fp16_scale_log2);
    a.h16_inv = std::ldexp(1.0f, dm->r.fp16_scale_log2);
    a.cd = make_coll<double>(dm->r);
    a.cf = make_coll<float>(dm->r);
    return a;
}

int need_bound(lbm_domain* dm)
{
    if (!dm) return fail(LBM_EINVAL, "domain is NULL");
    if (!dm->bound) return fail(LBM_ESTATE, "domain has no bound buffers (call lbm_bind)");
    return LBM_OK;
}

// The residual monitor's reference velocity restarts from zero whenever the
// state is replaced (initialisation, mask, populations written).
int clear_uprev(lbm_domain* dm)
{
    HIPCHK(hipMemsetAsync(dm->work + dm->L.uprev, 0, (size_t)3 * dm->L.npad * sizeof(double), dm->stream));
    return LBM_OK;
}

int64_t chunk_nodes(const lbm_domain* dm, size_t bytes_per_node)
{
    const size_t stage = dm->L.work - dm->L.stage;
    return std::max<int64_t>(1, std::min<int64_t>(dm->N, (int64_t)(stage / bytes_per_node)));
}

// Enqueue nsteps steps on stream st (the bound stream, or the capture
// stream while a graph is recorded), advancing the host-side state.
int run_steps(lbm_domain* dm, int64_t nsteps, hipStream_t st)
{
    StepArgs a = step_args(dm);
    if (a.ntiles > dm->L.max_parts)
        return fail(LBM_EINVAL, "tile %dx%dx%d gives %d tiles, more than the %lld monitor slots", dm->tx, dm->ty,
                    dm->tz, a.ntiles, (long long)dm->L.max_parts);
    // the population stride must cover every slot the layout addresses
    if ((dm->d.layout == LBM_DENSE && dm->S != dm->N) || (dm->d.layout == LBM_COMPACT && dm->S < dm->Nf) ||
        dm->S > dm->L.npad || (dm->d.layout == LBM_COMPACT && dm->tx != 64 && dm->tx != 128 && dm->tx != 256))
        return fail(LBM_ESTATE, "inconsistent population stride or tile for the layout");
    for (int64_t s = 0; s < nsteps; ++s) {
        int pat;
        if (dm->d.scheme == LBM_AB) {
            pat = PAT_AB;
            a.src = copy_ptr(dm, dm->cur);
            a.dst = copy_ptr(dm, 1 - dm->cur);
        } else {
            pat = dm->parity == 0 ? PAT_AA_PULL : PAT_AA_LOCAL;
            a.src = dm->pdf;
            a.dst = dm->pdf;
        }
        const bool mon = dm->mon_k > 0 && (dm->t % dm->mon_k) == 0;
        HIPCHK(launch_step(dm->d.lattice, kernel_op(dm->r) | (a.fallback ? OP_FB : 0), dm->d.precision, pat, mon,
                           dm->d.layout, a, st));
        if (mon) {
            // the compact slot kernels run one block per 256 fluid slots, the others one per tile
            const int64_t nparts = (dm->d.layout == LBM_COMPACT && (pat == PAT_AA_LOCAL || a.pull_slots))
                                       ? (dm->Nf + 255) / 256
                                       : a.ntiles;
            // the record goes to ring slot (device counter mod kHistory), so a
            // replayed graph fills consecutive slots
            HIPCHK(launch_finalize_ring((double*)dm->work, nparts, dm->work + dm->L.hist,
                                        (int64_t*)(dm->work + dm->L.counter), kHistory, dm->t, (double)dm->N, st));
            dm->hist_time[(size_t)(dm->hist_written % kHistory)] = dm->t;
            dm->hist_written++;
        }
        if (dm->d.scheme == LBM_AB) dm->cur = 1 - dm->cur;
        else dm->parity ^= 1;
        dm->t++;
    }
    return LBM_OK;
}

// The history restarts: host counters and the device ring counter.
int reset_history(lbm_domain* dm)
{
    dm->hist_written = dm->hist_read = 0;
    HIPCHK(launch_fill_u8((uint8_t*)(dm->work + dm->L.counter), sizeof(int64_t), 0, dm->stream));
    return LBM_OK;
}

void drop_graph(lbm_domain* dm)
{
    if (dm->graph) (void)hipGraphExecDestroy(dm->graph);
    dm->graph = nullptr;
}

// Capture graph_steps steps from the current (replay-start) state into a
// graph on a private stream; the host state is restored afterwards (a
// capture runs nothing).
int build_graph(lbm_domain* dm)
{
    drop_graph(dm);
    if (!dm->cap) HIPCHK(hipStreamCreateWithFlags(&dm->cap, hipStreamNonBlocking));
    const int64_t t = dm->t, hw = dm->hist_written;
    const int cur = dm->cur, parity = dm->parity;
    const std::vector<int64_t> times = dm->hist_time;
    HIPCHK(hipStreamBeginCapture(dm->cap, hipStreamCaptureModeThreadLocal));
    const int rc = run_steps(dm, dm->graph_steps, dm->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(dm->cap, &g);
    dm->t = t;
    dm->hist_written = hw;
    dm->cur = cur;
    dm->parity = parity;
    dm->hist_time = times;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(LBM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&dm->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        dm->graph = nullptr;
        return fail(LBM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
    }
    dm->graph_gen = dm->gen;
    return LBM_OK;
}

// Upload a host mask (nullptr = all fluid) in the domain's layout and set
// the population stride.
int upload_mask(lbm_domain* dm, const uint8_t* host_mask)
{
    dm->gen++;
    if (dm->d.layout == LBM_DENSE) {
        if (host_mask) {
            // stored as 0 / 1 bytes whatever nonzero value marks a solid
            std::vector<uint8_t> m((size_t)dm->N);
            int64_t nf = 0;
            for (int64_t n = 0; n < dm->N; ++n) {
                m[(size_t)n] = host_mask[n] ? 1 : 0;
                nf += host_mask[n] == 0;
            }
            HIPCHK(hipMemcpyAsync(dm->mask, m.data(), (size_t)dm->N, hipMemcpyHostToDevice, dm->stream));
            HIPCHK(hipStreamSynchronize(dm->stream));
            dm->Nf = nf;
        } else {
            HIPCHK(launch_fill_u8(dm->mask, dm->N, 0, dm->stream));
            dm->Nf = dm->N;
        }
        dm->S = dm->N;
        HIPCHK(hipStreamSynchronize(dm->stream));
        return LBM_OK;
    }
    int per[3];
    for (int k = 0; k < 3; ++k) per[k] = dm->d.periodic[k] ? 1 : 0;
    if (dm->D == 2) per[2] = 1;
    CompactMask cm;
    std::string err;
    if (!build_compact_mask(dm->d.nx, dm->d.ny, dm->d.nz, per, host_mask, cm, err)) return fail(LBM_EINVAL, "%s", err.c_str());
    dm->Nf = cm.fluid;
    dm->S = compact_stride(dm->Nf, prec_bytes(dm->d.precision));
    HIPCHK(hipMemcpyAsync(dm->mask + dm->L.bits_off, cm.bits.data(), cm.bits.size() * 8, hipMemcpyHostToDevice,
                          dm->stream));
    HIPCHK(hipMemcpyAsync(dm->mask + dm->L.base_off, cm.base.data(), cm.base.size() * 4, hipMemcpyHostToDevice,
                          dm->stream));
    if (!cm.wstart.empty())
        HIPCHK(hipMemcpyAsync(dm->mask + dm->L.wstart_off, cm.wstart.data(), cm.wstart.size() * 4,
                              hipMemcpyHostToDevice, dm->stream));
    HIPCHK(hipMemcpyAsync(dm->mask + dm->L.recs_off, cm.recs.data(), cm.recs.size() * sizeof(SegRec),
                          hipMemcpyHostToDevice, dm->stream));
    HIPCHK(hipStreamSynchronize(dm->stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

int lbm_lattice_info(int32_t lattice, int32_t* q, int32_t* c, double* w, int32_t* opp)
{
    auto fill = [&](auto L) {
        using LT = decltype(L);
        if (q) *q = LT::Q;
        for (int i = 0; i < LT::Q; ++i) {
            if (c) { c[3 * i] = LT::cx[i]; c[3 * i + 1] = LT::cy[i]; c[3 * i + 2] = LT::cz[i]; }
            if (w) w[i] = LT::w[i];
            if (opp) opp[i] = lbm::opp(i);
        }
        return LBM_OK;
    };
    switch (lattice) {
    case 0: return fill(Lattice<0>{});
    case 1: return fill(Lattice<1>{});
    case 2: return fill(Lattice<2>{});
    default: return fail(LBM_EINVAL, "unknown lattice %d", lattice);
    }
}

int lbm_query_sizes(const lbm_desc* desc, const lbm_rheology* rh, lbm_sizes* out)
{
    int rc = check_desc(desc);
    if (rc) return rc;
    if (rh && (rc = check_rheology(rh))) return rc;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    const Layout L = layout_of(desc, rh);
    out->pdf_bytes = L.pdf;
    out->tau_bytes = L.tau;
    out->mask_bytes = L.mask;
    out->work_bytes = L.work;
    return LBM_OK;
}

int lbm_create(const lbm_desc* desc, const lbm_rheology* rh, lbm_domain** out)
{
    int rc = check_desc(desc);
    if (rc) return rc;
    if ((rc = check_rheology(rh))) return rc;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    lbm_domain* dm = new (std::nothrow) lbm_domain();
    if (!dm) return fail(LBM_EINVAL, "host allocation failed");
    dm->d = *desc;
    dm->r = *rh;
    dm->Q = lattice_q(desc->lattice);
    dm->D = lattice_d(desc->lattice);
    dm->N = (int64_t)desc->nx * desc->ny * desc->nz;
    dm->L = layout_of(desc, rh);
    default_tile(dm);
    *out = dm;
    return LBM_OK;
}

int lbm_bind(lbm_domain* dm, void* pdf_dev, void* tau_dev, void* mask_dev, void* work_dev, void* hip_stream)
{
    if (!dm) return fail(LBM_EINVAL, "domain is NULL");
    if (!pdf_dev || !mask_dev || !work_dev) return fail(LBM_EINVAL, "pdf, mask and work buffers are required");
    if (dm->r.op == LBM_PR && !tau_dev) return fail(LBM_EINVAL, "the PR operator needs the tau buffer");
    if (((uintptr_t)pdf_dev | (uintptr_t)work_dev | (uintptr_t)(tau_dev ? tau_dev : pdf_dev)) % 16)
        return fail(LBM_EINVAL, "device buffers must be 16-byte aligned");
    dm->pdf = (char*)pdf_dev;
    dm->tau = tau_dev;
    dm->mask = (uint8_t*)mask_dev;
    dm->work = (char*)work_dev;
    dm->stream = (hipStream_t)hip_stream;
    // resolve this GPU's allocation-free monitor scratch now, at set-up, so
    // that lbm_monitors_async looks nothing up when it runs (e.g. under
    // graph capture)
    HIPCHK(scratch_partials(dm->stream, &dm->scratch));
    dm->bound = true;
    int rc = upload_mask(dm, nullptr);
    if (rc) return rc;
    const double zero[3] = {0, 0, 0};
    return lbm_init_equilibrium(dm, dm->r.rho0, zero);
}

int lbm_set_mask(lbm_domain* dm, const uint8_t* host_mask)
{
    int rc = need_bound(dm);
    if (rc) return rc;
    if (!host_mask) return fail(LBM_EINVAL, "host_mask is NULL");
    if ((rc = upload_mask(dm, host_mask))) return rc;
    const double zero[3] = {0, 0, 0};
    return lbm_init_equilibrium(dm, dm->r.rho0, zero);
}

int lbm_init_equilibrium(lbm_domain* dm, double rho0, const double* u0)
{
    int rc = need_bound(dm);
    if (rc) return rc;
    if (!(rho0 > 0)) return fail(LBM_EINVAL, "rho0 must be > 0");
    dm->cur = 0;
    dm->parity = 0;
    dm->t = 0;
    if ((rc = reset_history(dm))) return rc;
    NodeArgs a = node_args(dm);
    for (int k = 0; k < 3; ++k) a.u0[k] = u0 ? u0[k] : 0.0;
    HIPCHK(launch_init(dm->d.lattice, dm->r.op, dm->d.precision, a, rho0, dm->stream));
    return clear_uprev(dm);
}

int lbm_write_populations(lbm_domain* dm, const double* host_P, const double* host_tau)
{
    int rc = need_bound(dm);
    if (rc) return rc;
    if (!host_P) return fail(LBM_EINVAL, "host_P is NULL");
    if (dm->d.scheme == LBM_AA) dm->parity = 0;  // written as post-collision, swapped
    if ((rc = clear_uprev(dm))) return rc;
    const int Q = dm->Q;
    const int64_t chunk = chunk_nodes(dm, (size_t)(Q + 1) * 8);
    double* stage = (double*)(dm->work + dm->L.stage);
    for (int64_t n0 = 0; n0 < dm->N; n0 += chunk) {
        const int64_t cnt = std::min(chunk, dm->N - n0);
        HIPCHK(hipMemcpy2DAsync(stage, cnt * 8, host_P + n0, dm->N * 8, cnt * 8, Q, hipMemcpyHostToDevice, dm->stream));
        NodeArgs a = node_args(dm);
        a.tau = nullptr;
        if (host_tau && dm->tau) {
            HIPCHK(hipMemcpyAsync(stage + (size_t)Q * cnt, host_tau + n0, cnt * 8, hipMemcpyHostToDevice, dm->stream));
            a.tau = dm->tau;
        }
        a.out = stage;
        a.n0 = n0;
        a.count = cnt;
        HIPCHK(launch_pop_write(dm->d.lattice, dm->d.precision, a, dm->stream));
        HIPCHK(hipStreamSynchronize(dm->stream));
    }
    return LBM_OK;
}

int lbm_read_populations(lbm_domain* dm, double* host_P, double* host_tau)
{
    int rc = need_bound(dm);
    if (rc) return rc;
    if (!host_P) return fail(LBM_EINVAL, "host_P is NULL");
    const int Q = dm->Q;
    const int64_t chunk = chunk_nodes(dm, (size_t)(Q + 1) * 8);
    double* stage = (double*)(dm->work + dm->L.stage);
    for (int64_t n0 = 0; n0 < dm->N; n0 += chunk) {
        const int64_t cnt = std::min(chunk, dm->N - n0);
        NodeArgs a = node_args(dm);
        if (!(host_tau && dm->tau)) a.tau = nullptr;
        a.out = stage;
        a.n0 = n0;
        a.count = cnt;
        HIPCHK(launch_pop_read(dm->d.lattice, dm->d.precision, a, dm->stream));
        HIPCHK(hipMemcpy2DAsync(host_P + n0, dm->N * 8, stage, cnt * 8, cnt * 8, Q, hipMemcpyDeviceToHost, dm->stream));
        if (a.tau)
            HIPCHK(hipMemcpyAsync(host_tau + n0, stage + (size_t)Q * cnt, cnt * 8, hipMemcpyDeviceToHost, dm->stream));
        HIPCHK(hipStreamSynchronize(dm->stream));
    }
    return LBM_OK;
}

int lbm_step(lbm_domain* dm, int64_t nsteps)
{
    int rc = need_bound(dm);
    if (rc) return rc;
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    const int G = dm->graph_steps;
    while (nsteps > 0) {
        // a replay starts from the post-collision state in the first copy, at
        // a multiple of G, so that its monitor steps fall where they were
        // captured
        const bool at_start = dm->d.scheme == LBM_AA ? dm->parity == 0 : dm->cur == 0;
        const bool graph_ok = G > 0 && nsteps >= G && at_start && dm->t % G == 0 && (dm->mon_k == 0 || G % dm->mon_k == 0);
        if (!graph_ok) {
            int64_t n = nsteps;
            if (G > 0 && dm->t % G != 0) n = std::min<int64_t>(nsteps, G - dm->t % G);
            if ((rc = run_steps(dm, n, dm->stream))) return rc;
            nsteps -= n;
            continue;
        }
        if (!dm->graph || dm->graph_gen != dm->gen)
            if ((rc = build_graph(dm))) return rc;
        HIPCHK(hipGraphLaunch(dm->graph, dm->stream));
        for (int64_t k = 0; k < G; ++k) {
            if (dm->mon_k > 0 && (dm->t + k) % dm->mon_k == 0) {
                dm->hist_time[(size_t)(dm->hist_written % kHistory)] = dm->t + k;
                dm->hist_written++;
            }
        }
        dm->t += G;
        nsteps -= G;
    }
    return LBM_OK;
}

int lbm_set_graph_steps(lbm_domain* dm, int32_t steps)
{
    if (!dm) return fail(LBM_EINVAL, "domain is NULL");
    if (steps < 0 || (steps % 2)) return fail(LBM_EINVAL, "graph steps must be even and >= 0 (0 = no graph)");
    dm->graph_steps = steps;
    drop_graph(dm);
    return LBM_OK;
}

int lbm_time(lbm_domain* dm, int64_t* t)
{
    if (!dm || !t) return fail(LBM_EINVAL, "NULL argument");
    *t = dm->t;
    return LBM_OK;
}

int lbm_set_monitor_interval(lbm_domain* dm, int32_t k)
{
    if (!dm) return fail(LBM_EINVAL, "domain is NULL");
    if (k < 0) return fail(LBM_EINVAL, "interval must be >= 0");
    dm->mon_k = k;
    dm->gen++;
    return LBM_OK;
}

int lbm_read_history(lbm_domain* dm, lbm_monitor* out, int32_t max, int32_t* count)
{
    int rc = need_bound(dm);
    if (rc) return rc;
    if (!count || (max > 0 && !out)) return fail(LBM_EINVAL, "NULL argument");
    HIPCHK(hipStreamSynchronize(dm->stream));
    dm->hist_read = std::max(dm->hist_read, dm->hist_written - kHistory);
    const int64_t n = std::min<int64_t>(dm->hist_written - dm->hist_read, max);
    const MonitorRecord* ring = (const MonitorRecord*)(dm->work + dm->L.hist);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t slot = (dm->hist_read + k) % kHistory;
        HIPCHK(hipMemcpy(out + k, ring + slot, sizeof(MonitorRecord), hipMemcpyDeviceToHost));
        out[k].step = dm->hist_time[(size_t)slot];  // a replayed record carries its capture time
    }
    dm->hist_read += n;
    *count = (int32_t)n;
    return LBM_OK;
}

int lbm_monitors(lbm_domain* dm, lbm_monitor* out)
{
    int rc = need_bound(dm);
    if (rc) return rc;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    NodeArgs a = node_args(dm);
    a.n0 = 0;
    a.count = dm->N;
    a.reduce = 1;
    int64_t nb = 0;
    HIPCHK(launch_readout(dm->d.lattice, kernel_op(dm->r), dm->d.precision, a, dm->stream, &nb));
    char* rec = dm->work + dm->L.rec;
    HIPCHK(launch_finalize((double*)dm->work, nb, rec, dm->t, (double)dm->N, dm->stream));
    HIPCHK(hipMemcpyAsync(out, rec, sizeof(MonitorRecord), hipMemcpyDeviceToHost, dm->stream));
    HIPCHK(hipStreamSynchronize(dm->stream));
    if (out->nonfinite > 0) return fail(LBM_EUNSTABLE, "%lld non-finite fluid nodes at step %lld",
                                        (long long)out->nonfinite, (long long)out->step);
    if (out->umax > dm->umax_limit)
        return fail(LBM_EUNSTABLE, "max |u| = %g exceeds %g at step %lld", out->umax, dm->umax_limit,
                    (long long)out->step);
    return LBM_OK;
}

int lbm_monitors_async(lbm_domain* dm, void* record_dev)
{
    int rc = need_bound(dm);
    if (rc) return rc;
    if (!record_dev || (uintptr_t)record_dev % 8) return fail(LBM_EINVAL, "record_dev must be 8-byte aligned device memory");
    double* parts = dm->scratch;
    if (!parts) return fail(LBM_ESTATE, "no monitor scratch resolved for the bound stream");
    NodeArgs a = node_args(dm);
    a.n0 = 0;
    a.count = dm->N;
    a.reduce = 1;
    a.partials = parts;
    // at most kScratchBlocks blocks: larger domains are walked with a grid
    // stride, so the scratch always holds every block's partials
    int64_t nb = 0;
    HIPCHK(launch_readout(dm->d.lattice, kernel_op(dm->r), dm->d.precision, a, dm->stream, &nb, kScratchBlocks));
    HIPCHK(launch_finalize(parts, nb, record_dev, dm->t, (double)dm->N, dm->stream));
    return LBM_OK;
}

int lbm_set_umax_limit(lbm_domain* dm, double umax)
{
    if (!dm) return fail(LBM_EINVAL, "domain is NULL");
    if (!(umax > 0)) return fail(LBM_EINVAL, "umax limit must be > 0");
    dm->umax_limit = umax;
    return LBM_OK;
}

int lbm_read_moments(lbm_domain* dm, double* rho, double* u, double* nu_app, uint8_t* unyielded)
{
    int rc = need_bound(dm);
    if (rc) return rc;
    const int64_t chunk = chunk_nodes(dm, 5 * 8 + 1);
    double* stage = (double*)(dm->work + dm->L.stage);
    for (int64_t n0 = 0; n0 < dm->N; n0 += chunk) {
        const int64_t cnt = std::min(chunk, dm->N - n0);
        NodeArgs a = node_args(dm);
        a.out = stage;
        a.out_flags = (uint8_t*)(stage + 5 * cnt);
        a.n0 = n0;
        a.count = cnt;
        HIPCHK(launch_readout(dm->d.lattice, kernel_op(dm->r), dm->d.precision, a, dm->stream, nullptr));
        if (rho) HIPCHK(hipMemcpyAsync(rho + n0, stage, cnt * 8, hipMemcpyDeviceToHost, dm->stream));
        if (u)
            for (int k = 0; k < 3; ++k)
                HIPCHK(hipMemcpyAsync(u + (size_t)k * dm->N + n0, stage + (size_t)(1 + k) * cnt, cnt * 8,
                                      hipMemcpyDeviceToHost, dm->stream));
        if (nu_app) HIPCHK(hipMemcpyAsync(nu_app + n0, stage + 4 * cnt, cnt * 8, hipMemcpyDeviceToHost, dm->stream));
        if (unyielded)
            HIPCHK(hipMemcpyAsync(unyielded + n0, a.out_flags, cnt, hipMemcpyDeviceToHost, dm->stream));
        HIPCHK(hipStreamSynchronize(dm->stream));
    }
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// checkpoints (format and validation: host.hpp)
// ---------------------------------------------------------------------------
int lbm_save(lbm_domain* dm, void* blob, size_t* bytes)
{
    int rc = need_bound(dm);
    if (rc) return rc;
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    CkptHeader h{};
    memcpy(h.magic, kCkptMagic, 8);
    h.version = kCkptVersion;
    h.header_bytes = sizeof(CkptHeader);
    h.desc = dm->d;
    h.rh = dm->r;
    h.t = dm->t;
    h.stride = dm->S;
    h.fluid = dm->Nf;
    h.parity = dm->parity;
    h.q = dm->Q;
    checkpoint_sizes(dm->d, dm->r.op == LBM_PR, dm->S, h);
    const size_t need = sizeof(h) + h.pdf_bytes + h.tau_bytes + h.mask_bytes + h.uprev_bytes;
    if (!blob) {
        *bytes = need;
        return LBM_OK;
    }
    if (*bytes < need) return fail(LBM_EINVAL, "blob too small: %zu < %zu", *bytes, need);
    char* const payload = (char*)blob + sizeof h;
    char* p = payload;
    HIPCHK(hipStreamSynchronize(dm->stream));
    const char* src = dm->d.scheme == LBM_AB ? copy_ptr(dm, dm->cur) : dm->pdf;
    HIPCHK(hipMemcpy(p, src, h.pdf_bytes, hipMemcpyDeviceToHost));
    p += h.pdf_bytes;
    if (h.tau_bytes) HIPCHK(hipMemcpy(p, dm->tau, h.tau_bytes, hipMemcpyDeviceToHost));
    p += h.tau_bytes;
    // the dense mask bytes, or the compact layout's fluid bitmap (everything
    // else of the compact mask is rebuilt from it on load)
    HIPCHK(hipMemcpy(p, dm->mask + (dm->d.layout == LBM_DENSE ? 0 : dm->L.bits_off), h.mask_bytes,
                     hipMemcpyDeviceToHost));
    p += h.mask_bytes;
    // the residual monitor's reference velocity: components at 0, S, 2S
    HIPCHK(hipMemcpy(p, dm->work + dm->L.uprev, h.uprev_bytes, hipMemcpyDeviceToHost));
    h.checksum = checkpoint_checksum(h, payload, need - sizeof h);
    memcpy(blob, &h, sizeof h);
    *bytes = need;
    return LBM_OK;
}

int lbm_check_checkpoint(const lbm_desc* desc, const lbm_rheology* rh, const void* blob, size_t bytes)
{
    int rc = check_desc(desc);
    if (rc) return rc;
    if ((rc = check_rheology(rh))) return rc;
    if (!blob) return fail(LBM_EINVAL, "blob is NULL");
    CkptView v;
    std::string err;
    if ((rc = parse_checkpoint(*desc, rh->op == LBM_PR, blob, bytes, v, err))) return fail(rc, "%s", err.c_str());
    return LBM_OK;
}

int lbm_load(lbm_domain* dm, const void* blob, size_t bytes)
{
    int rc = need_bound(dm);
    if (rc) return rc;
    if (!blob) return fail(LBM_EINVAL, "blob is NULL");
    CkptView v;
    std::string err;
    // everything is checked on the host before the device is touched
    if ((rc = parse_checkpoint(dm->d, dm->r.op == LBM_PR, blob, bytes, v, err))) return fail(rc, "%s", err.c_str());
    std::vector<uint8_t> mask;
    checkpoint_mask(dm->d, v, mask);
    // the slot tables are rebuilt from the mask, never taken from the blob
    if ((rc = upload_mask(dm, mask.data()))) return rc;
    if (dm->Nf != v.h.fluid || dm->S != v.h.stride)
        return fail(LBM_EFORMAT, "checkpoint mask gives another fluid count or stride");
    dm->cur = 0;
    HIPCHK(hipMemcpy(dm->pdf, v.pdf, v.h.pdf_bytes, hipMemcpyHostToDevice));
    if (v.h.tau_bytes) HIPCHK(hipMemcpy(dm->tau, v.tau, v.h.tau_bytes, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dm->work + dm->L.uprev, v.uprev, v.h.uprev_bytes, hipMemcpyHostToDevice));
    dm->t = v.h.t;
    dm->parity = v.h.parity;
    return reset_history(dm);
}

// ---------------------------------------------------------------------------
// tiles
// ---------------------------------------------------------------------------
int lbm_set_tile(lbm_domain* dm, int32_t tx, int32_t ty, int32_t tz)
{
    if (!dm) return fail(LBM_EINVAL, "domain is NULL");
    int rc = check_tile(dm, tx, ty, tz);
    if (rc) return rc;
    dm->tx = tx;
    dm->ty = ty;
    dm->tz = tz;
    dm->gen++;
    return LBM_OK;
}

int lbm_set_tile_order(lbm_domain* dm, int32_t brick_rows, int32_t brick_planes)
{
    if (!dm) return fail(LBM_EINVAL, "domain is NULL");
    if (brick_rows < 0 || brick_planes < 0) return fail(LBM_EINVAL, "brick sizes must be >= 0 (0 = default)");
    dm->bry = brick_rows;
    dm->brz = brick_planes;
    dm->gen++;
    return LBM_OK;
}

int lbm_get_tile_order(lbm_domain* dm, int32_t* brick_rows, int32_t* brick_planes)
{
    if (!dm || !brick_rows || !brick_planes) return fail(LBM_EINVAL, "NULL argument");
    const int ntx = (dm->d.nx + dm->tx - 1) / dm->tx, nty = (dm->d.ny + dm->ty - 1) / dm->ty;
    const int ntz = (dm->d.nz + dm->tz - 1) / dm->tz;
    int bry = 0, brz = 0;
    tile_order(dm, ntx, nty, ntz, bry, brz);
    *brick_rows = bry;
    *brick_planes = brz;
    return LBM_OK;
}

int lbm_set_pull_form(lbm_domain* dm, int32_t form)
{
    if (!dm) return fail(LBM_EINVAL, "domain is NULL");
    if (form != LBM_PULL_AUTO && form != LBM_PULL_SLOTS && form != LBM_PULL_ROWS)
        return fail(LBM_EINVAL, "unknown pull form %d", (int)form);
    dm->pull_form = form;
    dm->gen++;
    return LBM_OK;
}

int lbm_get_pull_form(lbm_domain* dm, int32_t* form)
{
    if (!dm || !form) return fail(LBM_EINVAL, "NULL argument");
    *form = pull_slots(dm) ? LBM_PULL_SLOTS : LBM_PULL_ROWS;
    return LBM_OK;
}

int lbm_get_tile(lbm_domain* dm, int32_t* tx, int32_t* ty, int32_t* tz)
{
    if (!dm || !tx || !ty || !tz) return fail(LBM_EINVAL, "NULL argument");
    *tx = dm->tx;
    *ty = dm->ty;
    *tz = dm->tz;
    return LBM_OK;
}

int lbm_autotune(lbm_domain* dm, int32_t trial_steps)
{
    int rc = need_bound(dm);
    if (rc) return rc;
    if (trial_steps < 1) return fail(LBM_EINVAL, "trial_steps must be >= 1");
    // candidate shapes: wavefront-wide rows first, then squatter tiles
    static const int cand3[][3] = {{256, 1, 1}, {128, 2, 1}, {64, 4, 1}, {64, 2, 2}, {128, 1, 2},
                                   {32, 8, 1},  {32, 4, 2}, {64, 1, 4}, {16, 4, 4}, {64, 2, 1},
                                   {64, 1, 1},  {128, 1, 1}};
    static const int cand2[][3] = {{256, 1, 1}, {128, 2, 1}, {64, 4, 1}, {32, 8, 1}, {16, 16, 1},
                                   {8, 32, 1},  {4, 64, 1},  {64, 2, 1}, {64, 1, 1}, {128, 1, 1}};
    // save the state; trial steps run on it and it is restored afterwards
    size_t bytes = 0;
    if ((rc = lbm_save(dm, nullptr, &bytes))) return rc;
    std::vector<char> saved(bytes);
    if ((rc = lbm_save(dm, saved.data(), &bytes))) return rc;
    const int mon_k = dm->mon_k;
    dm->mon_k = 0;
    // Every exit below restores the monitor interval, tile and kernel form
    // and reloads the saved state; a HIP error is reported after that.
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    static const int candc3[][3] = {{64, 4, 1}, {64, 2, 2}, {64, 1, 4}, {128, 2, 1}, {128, 1, 2}, {256, 1, 1},
                                    {64, 2, 1}, {64, 1, 2}, {64, 1, 1}};
    static const int candc2[][3] = {{64, 4, 1}, {128, 2, 1}, {256, 1, 1}, {64, 2, 1}, {64, 1, 1}};
    const int (*cand)[3];
    int nc;
    if (dm->d.layout == LBM_COMPACT) {
        cand = dm->D == 3 ? candc3 : candc2;
        nc = dm->D == 3 ? (int)(sizeof candc3 / sizeof candc3[0]) : (int)(sizeof candc2 / sizeof candc2[0]);
    } else {
        cand = dm->D == 3 ? cand3 : cand2;
        nc = dm->D == 3 ? (int)(sizeof cand3 / sizeof cand3[0]) : (int)(sizeof cand2 / sizeof cand2[0]);
    }
    int best = -2;  // -1: the slot kernel (compact layout), c >= 0: row kernel with tile c
    float best_ms = 1e30f;
    const int keep[3] = {dm->tx, dm->ty, dm->tz};
    const int keep_form = dm->pull_form;
    for (int c = dm->d.layout == LBM_COMPACT ? -1 : 0; c < nc && he == hipSuccess; ++c) {
        if (c >= 0) {
            const int tx = cand[c][0], ty = cand[c][1], tz = cand[c][2];
            if (check_tile(dm, tx, ty, tz) != LBM_OK) continue;
            if (tx > 2 * pow2ceil(dm->d.nx) || ty > 2 * pow2ceil(dm->d.ny)) continue;
            dm->tx = tx;
            dm->ty = ty;
            dm->tz = tz;
        }
        dm->pull_form = c < 0 ? LBM_PULL_SLOTS : LBM_PULL_ROWS;
        if ((rc = run_steps(dm, 2, dm->stream))) break;
        if ((he = hipEventRecord(e0, dm->stream)) != hipSuccess) break;
        if ((rc = run_steps(dm, trial_steps, dm->stream))) break;
        if ((he = hipEventRecord(e1, dm->stream)) != hipSuccess) break;
        if ((he = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0;
        if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dm->mon_k = mon_k;
    dm->tx = keep[0];
    dm->ty = keep[1];
    dm->tz = keep[2];
    dm->pull_form = keep_form;
    const bool ok = rc == LBM_OK && he == hipSuccess;
    if (ok && best >= 0) {
        dm->tx = cand[best][0];
        dm->ty = cand[best][1];
        dm->tz = cand[best][2];
    }
    if (ok && best >= -1 && dm->d.layout == LBM_COMPACT) dm->pull_form = best < 0 ? LBM_PULL_SLOTS : LBM_PULL_ROWS;
    dm->gen++;
    const int rc_load = lbm_load(dm, saved.data(), bytes);
    if (he != hipSuccess) return fail(LBM_EHIP, "autotune: %s", hipGetErrorString(he));
    if (rc) return rc;
    return rc_load;
}

int lbm_destroy(lbm_domain* dm)
{
    if (!dm) return LBM_OK;
    if (dm->bound && dm->stream) (void)hipStreamSynchronize(dm->stream);
    drop_graph(dm);
    if (dm->cap) (void)hipStreamDestroy(dm->cap);
    delete dm;
    return LBM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched sweep
// ---------------------------------------------------------------------------
namespace {

constexpr int kBatchHistory = 256;

struct BatchLayout {
    size_t pdf, tau, sims, work_list, parts, recs, counter, uprev, stage, total;
};

}  // namespace

struct lbm_batch {
    int count = 0, lat = 0, prec = 0, Q = 0, D = 0;
    std::vector<lbm_desc> d;
    std::vector<lbm_rheology> r;
    std::vector<BatchSim> sims;
    std::vector<int> work;
    int nitems = 0;
    BatchLayout L{};
    bool bound = false;
    char* pdf = nullptr;
    char* tau = nullptr;
    char* workbuf = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    int parity = 0;
    int64_t t = 0;
    int mon_k = 0;
    std::vector<int64_t> mon_times;
    int64_t hist_read = 0;
    int graph_steps = 100;
    hipGraphExec_t graph = nullptr;
    int graph_for_mon = -1;
    int grid = 0;
    int policy = 3;  // tile policy: 0 fewest padded nodes (wide rows on ties), 1 prefer 64-wide rows, 2 fixed 64x4x1,
                     // 3 (default) runs of 256 consecutive nodes
    int xcd = 0;     // work-item order: 1 = one contiguous chunk per XCD, 0 (default) = plain grid stride
    size_t bound_total = 0;  // work-buffer bytes the layout had when bound
};

namespace {

void tile_for(const lbm_desc& d, int D, int policy, int& tx, int& ty, int& tz)
{
    static const int c3[][3] = {{256, 1, 1}, {128, 2, 1}, {64, 4, 1}, {64, 2, 2}, {32, 8, 1},
                                {32, 4, 2}, {16, 16, 1}, {16, 8, 2}, {16, 4, 4}};
    static const int c2[][3] = {{256, 1, 1}, {128, 2, 1}, {64, 4, 1}, {32, 8, 1}, {16, 16, 1}, {8, 32, 1}, {4, 64, 1}};
    const int (*c)[3] = D == 3 ? c3 : c2;
    const int nc = D == 3 ? 9 : 7;
    if (policy == 2) { tx = 64; ty = 4; tz = 1; return; }
    if (policy == 3) { tx = 256; ty = 1; tz = 1; return; }  // node runs: rows wrap, reported as 256 x 1 x 1
    int64_t best = -1;
    for (int k = 0; k < nc; ++k) {
        if (policy == 1 && c[k][0] < 64) continue;
        const int64_t pad = (int64_t)((d.nx + c[k][0] - 1) / c[k][0]) * c[k][0] * (int64_t)((d.ny + c[k][1] - 1) / c[k][1]) *
                            c[k][1] * (int64_t)((d.nz + c[k][2] - 1) / c[k][2]) * c[k][2];
        if (best < 0 || pad < best) { best = pad; tx = c[k][0]; ty = c[k][1]; tz = c[k][2]; }
    }
}

constexpr int kBatchPolicies = 4;

int64_t tiles_of(const lbm_desc& d, int D, int policy)
{
    if (policy == 3) return ((int64_t)d.nx * d.ny * d.nz + 255) / 256;
    int tx = 0, ty = 0, tz = 0;
    tile_for(d, D, policy, tx, ty, tz);
    return (int64_t)((d.nx + tx - 1) / tx) * ((d.ny + ty - 1) / ty) * ((d.nz + tz - 1) / tz);
}

// Work list and parameter table for the current tile policy.  The device
// layout (BatchLayout) is sized for the largest work list any policy gives,
// so it does not move when the autotuner switches policy.
int batch_plan(lbm_batch* b)
{
    b->sims.assign(b->count, BatchSim{});
    b->work.clear();
    int64_t off_pdf = 0, off_tau = 0, off_u = 0;
    for (int k = 0; k < b->count; ++k) {
        BatchSim& s = b->sims[k];
        const lbm_desc& d = b->d[k];
        s.nx = d.nx; s.ny = d.ny; s.nz = d.nz;
        for (int a = 0; a < 3; ++a) s.per[a] = d.periodic[a] ? 1 : 0;
        if (b->D == 2) s.per[2] = 1;
        s.op = b->r[k].op;
        tile_for(d, b->D, b->policy, s.tx, s.ty, s.tz);
        s.linear = b->policy == 3 ? 1 : 0;
        s.ntx = s.linear ? (int)tiles_of(d, b->D, 3) : (d.nx + s.tx - 1) / s.tx;
        s.nty = s.linear ? 1 : (d.ny + s.ty - 1) / s.ty;
        s.ntz = s.linear ? 1 : (d.nz + s.tz - 1) / s.tz;
        const int64_t items = (int64_t)s.ntx * s.nty * s.ntz;
        if ((int64_t)b->work.size() + items > INT32_MAX) return fail(LBM_EINVAL, "batch too large");
        s.item0 = (int)b->work.size();
        s.nitems = (int)items;
        for (int64_t j = 0; j < items; ++j) b->work.push_back(k);
        s.N = (int64_t)d.nx * d.ny * d.nz;
        s.S = (s.N + 63) / 64 * 64;
        s.off_pdf = off_pdf;
        s.off_tau = off_tau;
        s.off_u = off_u;
        off_pdf += s.S * b->Q;
        off_tau += s.S;
        off_u += 3 * s.S;
        s.cd = make_coll<double>(b->r[k]);
        s.cf = make_coll<float>(b->r[k]);
    }
    b->nitems = (int)b->work.size();
    int64_t cap = 0;
    for (int pol = 0; pol < kBatchPolicies; ++pol) {
        int64_t items = 0;
        for (int k = 0; k < b->count; ++k) items += tiles_of(b->d[k], b->D, pol);
        cap = std::max(cap, items);
    }
    if (cap > INT32_MAX) return fail(LBM_EINVAL, "batch too large");
    BatchLayout& L = b->L;
    L.pdf = align_up((size_t)off_pdf * prec_bytes(b->prec));
    bool any_pr = false;
    for (auto& r : b->r) any_pr |= r.op == LBM_PR;
    L.tau = any_pr ? align_up((size_t)off_tau * (b->prec == LBM_FP64 ? 8 : 4)) : 0;
    L.sims = 0;
    L.work_list = align_up(sizeof(BatchSim) * b->count);
    L.parts = L.work_list + align_up(sizeof(int) * (size_t)cap);
    L.recs = L.parts + align_up((size_t)cap * MP_COUNT * sizeof(double));
    L.counter = L.recs + align_up((size_t)kBatchHistory * b->count * sizeof(MonitorRecord));
    L.uprev = L.counter + kAlign;
    L.stage = L.uprev + align_up((size_t)off_u * sizeof(double));
    int64_t maxN = 0;
    for (auto& s : b->sims) maxN = std::max(maxN, s.N);
    size_t stage = std::min(kStageMax, align_up((size_t)maxN * (b->Q + 1) * 8));
    stage = std::max(stage, align_up((size_t)(b->Q + 1) * 8 * 256));
    L.total = L.stage + stage;
    // the bound buffers were sized for this layout; it must not change
    if (b->bound && L.total != b->bound_total) return fail(LBM_ESTATE, "batch layout changed after binding");
    return LBM_OK;
}

// Persistent grid: up to 4096 blocks (16 per CU), a multiple of 8 in the
// per-XCD order.
void batch_set_grid(lbm_batch* b)
{
    int g = std::max(1, std::min(b->nitems, 4096));
    if (b->xcd) g = (g + 7) / 8 * 8;
    b->grid = g;
}

int batch_need(lbm_batch* b)
{
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (!b->bound) return fail(LBM_ESTATE, "batch has no bound buffers (call lbm_batch_bind)");
    return LBM_OK;
}

BatchArgs batch_args(lbm_batch* b)
{
    BatchArgs a{};
    a.sims = (const BatchSim*)(b->workbuf + b->L.sims);
    a.work = (const int*)(b->workbuf + b->L.work_list);
    a.nitems = b->nitems;
    a.nsims = b->count;
    a.pdf = b->pdf;
    a.tau = b->tau;
    a.partials = (double*)(b->workbuf + b->L.parts);
    a.uprev = (double*)(b->workbuf + b->L.uprev);
    a.h16_scale = std::ldexp(1.0f, -b->r[0].fp16_scale_log2);
    a.h16_inv = std::ldexp(1.0f, b->r[0].fp16_scale_log2);
    a.fallback = (b->prec != LBM_FP64 && b->r[0].fp64_fallback) ? 1 : 0;
    a.xcd_chunks = b->xcd;
    return a;
}

// Enqueue nsteps steps on stream s (eagerly or while s is being captured).
int batch_enqueue(lbm_batch* b, int64_t nsteps, hipStream_t s, int& parity, int64_t& t, bool record_times)
{
    BatchArgs a = batch_args(b);
    for (int64_t k = 0; k < nsteps; ++k) {
        const int pat = parity == 0 ? PAT_AA_PULL : PAT_AA_LOCAL;
        const bool mon = b->mon_k > 0 && (t % b->mon_k) == 0;
        HIPCHK(launch_batch_step(b->lat, b->prec, pat, mon, a, b->grid, s));
        if (mon) {
            HIPCHK(launch_batch_finalize(a, nullptr, b->workbuf + b->L.recs, (const int64_t*)(b->workbuf + b->L.counter),
                                         t, kBatchHistory, s));
            HIPCHK(launch_batch_tick((int64_t*)(b->workbuf + b->L.counter), s));
            if (record_times) b->mon_times.push_back(t);
        }
        parity ^= 1;
        ++t;
    }
    return LBM_OK;
}

void batch_drop_graph(lbm_batch* b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->graph_for_mon = -1;
}

// Capture graph_steps steps starting at parity 0 and a time that is a
// multiple of graph_steps (so monitor steps fall at the same offsets).
int batch_build_graph(lbm_batch* b)
{
    batch_drop_graph(b);
    if (!b->cap) HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    int parity = 0;
    int64_t t = 0;
    int rc = batch_enqueue(b, b->graph_steps, b->cap, parity, t, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(LBM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        b->graph = nullptr;
        return fail(LBM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
    }
    b->graph_for_mon = b->mon_k;
    return LBM_OK;
}

NodeArgs batch_node_args(lbm_batch* b, int k)
{
    const BatchSim& s = b->sims[k];
    NodeArgs a{};
    a.pdf = b->pdf + (size_t)s.off_pdf * prec_bytes(b->prec);
    a.tau = b->tau ? (void*)(b->tau + (size_t)s.off_tau * (b->prec == LBM_FP64 ? 8 : 4)) : nullptr;
    if (b->r[k].op != LBM_PR) a.tau = nullptr;
    a.mask = nullptr;
    a.partials = (double*)(b->workbuf + b->L.parts);
    a.uprev = (const double*)(b->workbuf + b->L.uprev) + s.off_u;
    a.N = s.N;
    a.S = s.S;
    a.nx = s.nx; a.ny = s.ny; a.nz = s.nz;
    for (int q = 0; q < 3; ++q) a.per[q] = s.per[q];
    a.layout = b->parity == 0 ? 1 : 2;
    a.compact = 0;
    a.h16_scale = std::ldexp(1.0f, -b->r[k].fp16_scale_log2);
    a.h16_inv = std::ldexp(1.0f, b->r[k].fp16_scale_log2);
    a.cd = make_coll<double>(b->r[k]);
    a.cf = make_coll<float>(b->r[k]);
    return a;
}

int batch_check_sim(lbm_batch* b, int32_t sim)
{
    int rc = batch_need(b);
    if (rc) return rc;
    if (sim < 0 || sim >= b->count) return fail(LBM_EINVAL, "simulation index %d outside 0..%d", sim, b->count - 1);
    return LBM_OK;
}

int batch_validate(const lbm_desc* descs, const lbm_rheology* rh, int32_t count)
{
    if (!descs || !rh || count < 1) return fail(LBM_EINVAL, "need count >= 1 descriptors and rheologies");
    for (int k = 0; k < count; ++k) {
        int rc = check_desc(&descs[k]);
        if (rc) return fail(rc, "simulation %d: %s", k, g_err.c_str());
        if ((rc = check_rheology(&rh[k]))) return fail(rc, "simulation %d: %s", k, g_err.c_str());
        if (descs[k].lattice != descs[0].lattice || descs[k].precision != descs[0].precision)
            return fail(LBM_EINVAL, "all simulations of a batch share one lattice and one precision");
        if (descs[k].scheme != LBM_AA) return fail(LBM_EINVAL, "batches use the AA scheme");
        if (rh[k].op != LBM_PR && rh[k].op != LBM_IR)
            return fail(LBM_EINVAL, "simulation %d: batches take the PR and IR operators", k);
        if (rh[k].mrt_bulk > 0 || rh[k].mrt_even > 0)
            return fail(LBM_EINVAL, "simulation %d: batches use the TRT base collision (no MRT rates)", k);
        if (((int64_t)descs[k].nx * descs[k].ny * descs[k].nz + 63) / 64 * 64 * lattice_q(descs[k].lattice) >=
            ((int64_t)1 << 31))
            return fail(LBM_EINVAL, "simulation %d: batched simulations need Q * nodes < 2^31", k);
        if (rh[k].fp64_fallback != rh[0].fp64_fallback || rh[k].fp16_scale_log2 != rh[0].fp16_scale_log2)
            return fail(LBM_EINVAL, "all simulations of a batch share the fallback flag and the FP16 scale");
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_query_sizes(const lbm_desc* descs, const lbm_rheology* rh, int32_t count, lbm_sizes* out)
{
    int rc = batch_validate(descs, rh, count);
    if (rc) return rc;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    lbm_batch tmp;
    tmp.count = count;
    tmp.lat = descs[0].lattice;
    tmp.prec = descs[0].precision;
    tmp.Q = lattice_q(tmp.lat);
    tmp.D = lattice_d(tmp.lat);
    tmp.d.assign(descs, descs + count);
    tmp.r.assign(rh, rh + count);
    if ((rc = batch_plan(&tmp))) return rc;
    out->pdf_bytes = tmp.L.pdf;
    out->tau_bytes = tmp.L.tau;
    out->mask_bytes = 0;
    out->work_bytes = tmp.L.total;
    return LBM_OK;
}

int lbm_batch_create(const lbm_desc* descs, const lbm_rheology* rh, int32_t count, lbm_batch** out)
{
    int rc = batch_validate(descs, rh, count);
    if (rc) return rc;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return fail(LBM_EINVAL, "host allocation failed");
    b->count = count;
    b->lat = descs[0].lattice;
    b->prec = descs[0].precision;
    b->Q = lattice_q(b->lat);
    b->D = lattice_d(b->lat);
    b->d.assign(descs, descs + count);
    b->r.assign(rh, rh + count);
    if ((rc = batch_plan(b))) {
        delete b;
        return rc;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_bind(lbm_batch* b, void* pdf_dev, void* tau_dev, void* work_dev, void* hip_stream)
{
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (!pdf_dev || !work_dev || (b->L.tau && !tau_dev)) return fail(LBM_EINVAL, "missing device buffer");
    if (((uintptr_t)pdf_dev | (uintptr_t)work_dev | (uintptr_t)(tau_dev ? tau_dev : pdf_dev)) % 16)
        return fail(LBM_EINVAL, "device buffers must be 16-byte aligned");
    b->pdf = (char*)pdf_dev;
    b->tau = (char*)tau_dev;
    b->workbuf = (char*)work_dev;
    b->stream = (hipStream_t)hip_stream;
    b->bound = true;
    b->bound_total = b->L.total;
    batch_set_grid(b);
    batch_drop_graph(b);
    HIPCHK(hipMemcpyAsync(b->workbuf + b->L.sims, b->sims.data(), sizeof(BatchSim) * b->count, hipMemcpyHostToDevice,
                          b->stream));
    HIPCHK(hipMemcpyAsync(b->workbuf + b->L.work_list, b->work.data(), sizeof(int) * b->nitems, hipMemcpyHostToDevice,
                          b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return lbm_batch_init_equilibrium(b);
}

int lbm_batch_init_equilibrium(lbm_batch* b)
{
    int rc = batch_need(b);
    if (rc) return rc;
    b->parity = 0;
    b->t = 0;
    b->mon_times.clear();
    b->hist_read = 0;
    HIPCHK(hipMemsetAsync(b->workbuf + b->L.counter, 0, sizeof(int64_t), b->stream));
    HIPCHK(hipMemsetAsync(b->workbuf + b->L.uprev, 0, b->L.stage - b->L.uprev, b->stream));
    for (int k = 0; k < b->count; ++k) {
        NodeArgs a = batch_node_args(b, k);
        HIPCHK(launch_init(b->lat, b->r[k].op, b->prec, a, b->r[k].rho0, b->stream));
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    return LBM_OK;
}

int lbm_batch_write_populations(lbm_batch* b, int32_t sim, const double* host_P, const double* host_tau)
{
    int rc = batch_check_sim(b, sim);
    if (rc) return rc;
    if (!host_P) return fail(LBM_EINVAL, "host_P is NULL");
    if (b->parity != 0) return fail(LBM_ESTATE, "write populations only between step pairs (even time)");
    const BatchSim& s = b->sims[sim];
    HIPCHK(hipMemsetAsync(b->workbuf + b->L.uprev + (size_t)s.off_u * sizeof(double), 0,
                          (size_t)3 * s.S * sizeof(double), b->stream));
    const int Q = b->Q;
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(s.N, (int64_t)((b->L.total - b->L.stage) / ((Q + 1) * 8))));
    double* stage = (double*)(b->workbuf + b->L.stage);
    for (int64_t n0 = 0; n0 < s.N; n0 += chunk) {
        const int64_t cnt = std::min(chunk, s.N - n0);
        HIPCHK(hipMemcpy2DAsync(stage, cnt * 8, host_P + n0, s.N * 8, cnt * 8, Q, hipMemcpyHostToDevice, b->stream));
        NodeArgs a = batch_node_args(b, sim);
        if (!(host_tau && a.tau)) a.tau = nullptr;
        else HIPCHK(hipMemcpyAsync(stage + (size_t)Q * cnt, host_tau + n0, cnt * 8, hipMemcpyHostToDevice, b->stream));
        a.out = stage;
        a.n0 = n0;
        a.count = cnt;
        HIPCHK(launch_pop_write(b->lat, b->prec, a, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
    }
    return LBM_OK;
}

int lbm_batch_read_populations(lbm_batch* b, int32_t sim, double* host_P, double* host_tau)
{
    int rc = batch_check_sim(b, sim);
    if (rc) return rc;
    if (!host_P) return fail(LBM_EINVAL, "host_P is NULL");
    const BatchSim& s = b->sims[sim];
    const int Q = b->Q;
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(s.N, (int64_t)((b->L.total - b->L.stage) / ((Q + 1) * 8))));
    double* stage = (double*)(b->workbuf + b->L.stage);
    for (int64_t n0 = 0; n0 < s.N; n0 += chunk) {
        const int64_t cnt = std::min(chunk, s.N - n0);
        NodeArgs a = batch_node_args(b, sim);
        if (!host_tau) a.tau = nullptr;
        a.out = stage;
        a.n0 = n0;
        a.count = cnt;
        HIPCHK(launch_pop_read(b->lat, b->prec, a, b->stream));
        HIPCHK(hipMemcpy2DAsync(host_P + n0, s.N * 8, stage, cnt * 8, cnt * 8, Q, hipMemcpyDeviceToHost, b->stream));
        if (a.tau)
            HIPCHK(hipMemcpyAsync(host_tau + n0, stage + (size_t)Q * cnt, cnt * 8, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
    }
    return LBM_OK;
}

int lbm_batch_read_moments(lbm_batch* b, int32_t sim, double* rho, double* u, double* nu_app, uint8_t* unyielded)
{
    int rc = batch_check_sim(b, sim);
    if (rc) return rc;
    const BatchSim& s = b->sims[sim];
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(s.N, (int64_t)((b->L.total - b->L.stage) / 41)));
    double* stage = (double*)(b->workbuf + b->L.stage);
    for (int64_t n0 = 0; n0 < s.N; n0 += chunk) {
        const int64_t cnt = std::min(chunk, s.N - n0);
        NodeArgs a = batch_node_args(b, sim);
        a.out = stage;
        a.out_flags = (uint8_t*)(stage + 5 * cnt);
        a.n0 = n0;
        a.count = cnt;
        HIPCHK(launch_readout(b->lat, b->r[sim].op, b->prec, a, b->stream, nullptr));
        if (rho) HIPCHK(hipMemcpyAsync(rho + n0, stage, cnt * 8, hipMemcpyDeviceToHost, b->stream));
        if (u)
            for (int k = 0; k < 3; ++k)
                HIPCHK(hipMemcpyAsync(u + (size_t)k * s.N + n0, stage + (size_t)(1 + k) * cnt, cnt * 8,
                                      hipMemcpyDeviceToHost, b->stream));
        if (nu_app) HIPCHK(hipMemcpyAsync(nu_app + n0, stage + 4 * cnt, cnt * 8, hipMemcpyDeviceToHost, b->stream));
        if (unyielded) HIPCHK(hipMemcpyAsync(unyielded + n0, a.out_flags, cnt, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
    }
    return LBM_OK;
}

int lbm_batch_set_monitor_interval(lbm_batch* b, int32_t k)
{
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (k < 0) return fail(LBM_EINVAL, "interval must be >= 0");
    b->mon_k = k;
    return LBM_OK;
}

int lbm_batch_set_graph_steps(lbm_batch* b, int32_t steps)
{
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (steps < 0 || (steps % 2)) return fail(LBM_EINVAL, "graph steps must be even and >= 0 (0 = no graph)");
    b->graph_steps = steps;
    batch_drop_graph(b);
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int64_t nsteps)
{
    int rc = batch_need(b);
    if (rc) return rc;
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    const int G = b->graph_steps;
    while (nsteps > 0) {
        const bool graph_ok = G > 0 && nsteps >= G && b->parity == 0 && (b->t % G) == 0 &&
                              (b->mon_k == 0 || (G % b->mon_k) == 0);
        if (!graph_ok) {
            // eager steps up to the next point where a replay can start
            int64_t n = 1;
            if (G > 0 && (b->t % G) != 0) n = std::min<int64_t>(nsteps, G - b->t % G);
            else if (G == 0 || nsteps < G || (b->mon_k && G % b->mon_k)) n = nsteps;
            if ((rc = batch_enqueue(b, n, b->stream, b->parity, b->t, true))) return rc;
            nsteps -= n;
            continue;
        }
        if (!b->graph || b->graph_for_mon != b->mon_k)
            if ((rc = batch_build_graph(b))) return rc;
        HIPCHK(hipGraphLaunch(b->graph, b->stream));
        if (b->mon_k > 0)
            for (int64_t k = 0; k < G; k += b->mon_k) b->mon_times.push_back(b->t + k);
        b->t += G;
        nsteps -= G;
    }
    return LBM_OK;
}

int lbm_batch_time(lbm_batch* b, int64_t* t)
{
    if (!b || !t) return fail(LBM_EINVAL, "NULL argument");
    *t = b->t;
    return LBM_OK;
}

int lbm_batch_read_history(lbm_batch* b, lbm_monitor* out, int32_t max_records, int32_t* nrecords)
{
    int rc = batch_need(b);
    if (rc) return rc;
    if (!nrecords || (max_records > 0 && !out)) return fail(LBM_EINVAL, "NULL argument");
    HIPCHK(hipStreamSynchronize(b->stream));
    const int64_t written = (int64_t)b->mon_times.size();
    b->hist_read = std::max(b->hist_read, written - kBatchHistory);
    const int64_t n = std::min<int64_t>(written - b->hist_read, max_records);
    const MonitorRecord* ring = (const MonitorRecord*)(b->workbuf + b->L.recs);
    for (int64_t j = 0; j < n; ++j) {
        const int64_t c = b->hist_read + j;
        HIPCHK(hipMemcpy(out + j * b->count, ring + (c % kBatchHistory) * b->count, sizeof(MonitorRecord) * b->count,
                         hipMemcpyDeviceToHost));
        for (int k = 0; k < b->count; ++k) out[j * b->count + k].step = b->mon_times[c];
    }
    b->hist_read += n;
    *nrecords = (int32_t)n;
    return LBM_OK;
}

int lbm_batch_monitors(lbm_batch* b, lbm_monitor* out)
{
    int rc = batch_need(b);
    if (rc) return rc;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    for (int k = 0; k < b->count; ++k) {
        NodeArgs a = batch_node_args(b, k);
        a.n0 = 0;
        a.count = b->sims[k].N;
        a.reduce = 1;
        int64_t nb = 0;
        HIPCHK(launch_readout(b->lat, b->r[k].op, b->prec, a, b->stream, &nb));
        // the on-demand record lives after the history ring's counter
        char* rec = b->workbuf + b->L.counter + 64;
        HIPCHK(launch_finalize(a.partials, nb, rec, b->t, (double)b->sims[k].N, b->stream));
        HIPCHK(hipMemcpyAsync(out + k, rec, sizeof(MonitorRecord), hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
    }
    return LBM_OK;
}

int lbm_batch_get_tiles(lbm_batch* b, int32_t* tiles)
{
    if (!b || !tiles) return fail(LBM_EINVAL, "NULL argument");
    for (int k = 0; k < b->count; ++k) {
        tiles[3 * k] = b->sims[k].tx;
        tiles[3 * k + 1] = b->sims[k].ty;
        tiles[3 * k + 2] = b->sims[k].tz;
    }
    return LBM_OK;
}

int lbm_batch_set_schedule(lbm_batch* b, int32_t tile_policy, int32_t xcd_order)
{
    int rc = batch_need(b);
    if (rc) return rc;
    if (tile_policy < 0 || tile_policy >= kBatchPolicies || (xcd_order != 0 && xcd_order != 1))
        return fail(LBM_EINVAL, "tile policy must be 0..%d and the work-item order 0 or 1", kBatchPolicies - 1);
    HIPCHK(hipStreamSynchronize(b->stream));
    b->policy = tile_policy;
    b->xcd = xcd_order;
    if ((rc = batch_plan(b))) return rc;
    HIPCHK(hipMemcpy(b->workbuf + b->L.sims, b->sims.data(), sizeof(BatchSim) * b->count, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->workbuf + b->L.work_list, b->work.data(), sizeof(int) * b->nitems, hipMemcpyHostToDevice));
    batch_set_grid(b);
    batch_drop_graph(b);
    return LBM_OK;
}

int lbm_batch_get_schedule(lbm_batch* b, int32_t* tile_policy, int32_t* xcd_order)
{
    if (!b || !tile_policy || !xcd_order) return fail(LBM_EINVAL, "NULL argument");
    *tile_policy = b->policy;
    *xcd_order = b->xcd;
    return LBM_OK;
}

int lbm_batch_autotune(lbm_batch* b, int32_t trial_steps)
{
    int rc = batch_need(b);
    if (rc) return rc;
    if (trial_steps < 2 || (trial_steps % 2)) return fail(LBM_EINVAL, "trial_steps must be even and >= 2");
    HIPCHK(hipStreamSynchronize(b->stream));
    // save the state (populations and relaxation times); trial steps run on it
    std::vector<char> pdf(b->L.pdf), tau(b->L.tau);
    HIPCHK(hipMemcpy(pdf.data(), b->pdf, b->L.pdf, hipMemcpyDeviceToHost));
    if (b->L.tau) HIPCHK(hipMemcpy(tau.data(), b->tau, b->L.tau, hipMemcpyDeviceToHost));
    const int parity = b->parity, mon_k = b->mon_k, keep = b->policy + kBatchPolicies * b->xcd;
    const int64_t t = b->t;
    const auto times = b->mon_times;
    b->mon_k = 0;
    // A HIP error stops the trials; the schedule, the state and the monitor
    // settings are restored below before it is reported.
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    int best = keep;
    float best_ms = 1e30f;
    // candidates: tile policy x work-item order
    for (int cand = 0; cand < 2 * kBatchPolicies && rc == LBM_OK && he == hipSuccess; ++cand) {
        b->policy = cand % kBatchPolicies;
        b->xcd = cand / kBatchPolicies;
        if ((rc = batch_plan(b))) break;
        if ((he = hipMemcpy(b->workbuf + b->L.sims, b->sims.data(), sizeof(BatchSim) * b->count,
                            hipMemcpyHostToDevice)) != hipSuccess)
            break;
        if ((he = hipMemcpy(b->workbuf + b->L.work_list, b->work.data(), sizeof(int) * b->nitems,
                            hipMemcpyHostToDevice)) != hipSuccess)
            break;
        batch_set_grid(b);
        int par = b->parity;
        int64_t tt = b->t;
        if ((rc = batch_enqueue(b, 2, b->stream, par, tt, false))) break;
        if ((he = hipEventRecord(e0, b->stream)) != hipSuccess) break;
        if ((rc = batch_enqueue(b, trial_steps, b->stream, par, tt, false))) break;
        if ((he = hipEventRecord(e1, b->stream)) != hipSuccess) break;
        if ((he = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0;
        if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        if (ms < best_ms) {
            best_ms = ms;
            best = cand;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc != LBM_OK || he != hipSuccess) best = keep;
    b->policy = best % kBatchPolicies;
    b->xcd = best / kBatchPolicies;
    int rc2 = batch_plan(b);
    if (rc2 == LBM_OK) {
        HIPCHK(hipMemcpy(b->workbuf + b->L.sims, b->sims.data(), sizeof(BatchSim) * b->count, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->workbuf + b->L.work_list, b->work.data(), sizeof(int) * b->nitems, hipMemcpyHostToDevice));
        batch_set_grid(b);
    }
    HIPCHK(hipMemcpy(b->pdf, pdf.data(), b->L.pdf, hipMemcpyHostToDevice));
    if (b->L.tau) HIPCHK(hipMemcpy(b->tau, tau.data(), b->L.tau, hipMemcpyHostToDevice));
    b->parity = parity;
    b->t = t;
    b->mon_k = mon_k;
    b->mon_times = times;
    batch_drop_graph(b);
    if (he != hipSuccess) return fail(LBM_EHIP, "batch autotune: %s", hipGetErrorString(he));
    return rc ? rc : rc2;
}

int lbm_batch_destroy(lbm_batch* b)
{
    if (!b) return LBM_OK;
    if (b->bound && b->stream) (void)hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return LBM_OK;
}

}  // extern "C"
