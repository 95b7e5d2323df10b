// host.cpp -- host-side builders and the checkpoint format (see host.hpp).
#include "host.hpp"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

namespace lbm {

const char kCkptMagic[8] = {'L', 'B', 'M', 'C', 'K', 'P', 'T', '1'};

namespace {
int invalid(std::string& err, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int invalid(std::string& err, const char* fmt, ...)
{
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return LBM_EINVAL;
}
}  // namespace

int validate_desc(const lbm_desc* d, std::string& err)
{
    if (!d) return invalid(err, "descriptor is NULL");
    if (lattice_q(d->lattice) < 0) return invalid(err, "unknown lattice %d", d->lattice);
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return invalid(err, "non-positive size %dx%dx%d", d->nx, d->ny, d->nz);
    if (d->lattice == LBM_D2Q9 && d->nz != 1) return invalid(err, "D2Q9 needs nz == 1");
    if ((int64_t)d->nx * d->ny * d->nz > (int64_t)1 << 36) return invalid(err, "domain too large");
    if (d->precision < LBM_FP64 || d->precision > LBM_FP16) return invalid(err, "unknown precision %d", d->precision);
    if (d->scheme != LBM_AB && d->scheme != LBM_AA) return invalid(err, "unknown scheme %d", d->scheme);
    if (d->layout != LBM_COMPACT && d->layout != LBM_DENSE) return invalid(err, "unknown layout %d", d->layout);
    return LBM_OK;
}

int validate_rheology(const lbm_rheology* r, std::string& err)
{
    if (!r) return invalid(err, "rheology is NULL");
    if (r->op != LBM_PR && r->op != LBM_IR && r->op != LBM_PRI && r->op != LBM_IRHB)
        return invalid(err, "unknown operator %d", r->op);
    if (r->op == LBM_IRHB && !(r->hb_n >= 0.2 && r->hb_n <= 5.0))
        return invalid(err, "hb_n (flow index) must lie in [0.2, 5]");
    if (!(r->nu_p > 0)) return invalid(err, "nu_p must be > 0 (tau > 1/2)");
    if (!(r->sigma_y >= 0)) return invalid(err, "sigma_y must be >= 0");
    if (!(r->rho0 > 0)) return invalid(err, "rho0 must be > 0");
    for (int a = 0; a < 3; ++a)
        if (!isfinite(r->g[a])) return invalid(err, "body force must be finite");
    if (r->op == LBM_PR || r->op == LBM_PRI) {
        if (!(r->m >= 0)) return invalid(err, "m must be >= 0");
        if (!(r->gamma_c > 0)) return invalid(err, "gamma_c must be > 0");
        if (!(r->lambda_trt > 0)) return invalid(err, "lambda_trt must be > 0");
    }
    if (r->fp16_scale_log2 < 0 || r->fp16_scale_log2 > 24) return invalid(err, "fp16_scale_log2 outside 0..24");
    if (!(r->fallback_band >= 0)) return invalid(err, "fallback_band must be >= 0");
    if (r->flow_axis < 0 || r->flow_axis > 3) return invalid(err, "flow_axis must be 0 (off) or 1..3");
    if (!(r->mrt_bulk >= 0 && r->mrt_bulk < 2) || !(r->mrt_even >= 0 && r->mrt_even < 2))
        return invalid(err, "MRT rates must lie in [0, 2) (0: the shear rate)");
    if ((r->mrt_bulk > 0 || r->mrt_even > 0) && (r->op == LBM_IR || r->op == LBM_IRHB))
        return invalid(err, "the MRT base collision applies to the PR operators");
    if (r->mrt_bulk > 0 && r->op == LBM_PRI)
        return invalid(err, "PRI takes no separate MRT bulk rate (its tau solve scales the whole strain rate)");
    return LBM_OK;
}

int64_t compact_stride(int64_t nf, size_t elem_bytes)
{
    const int64_t S = std::max<int64_t>(64, (nf + 63) / 64 * 64);
    const int64_t P = 65536 / (int64_t)elem_bytes;  // 64 KiB in elements
    const int64_t r = S % P;
    if (r >= P / 4 && r < 3 * P / 4) return S;
    return S + ((P / 4 - r) % P + P) % P;
}

bool build_compact_mask(int nx, int ny, int nz, const int per[3], const uint8_t* mask, CompactMask& out,
                        std::string& err)
{
    const int W = (nx + 63) / 64;
    const int64_t rows = (int64_t)ny * nz;
    out.W = W;
    out.bits.assign((size_t)(rows * W), 0);
    out.base.assign((size_t)(rows * W), 0);
    out.wstart.clear();
    out.wstart.reserve((size_t)(rows * W + 1));
    uint64_t count = 0;
    for (int64_t r = 0; r < rows; ++r) {
        for (int w = 0; w < W; ++w) {
            uint64_t word = 0;
            for (int b = 0; b < 64; ++b) {
                const int x = 64 * w + b;
                if (x < nx && (!mask || mask[r * nx + x] == 0)) word |= 1ull << b;
            }
            out.bits[(size_t)(r * W + w)] = word;
            out.base[(size_t)(r * W + w)] = (uint32_t)count;
            count += (uint64_t)__builtin_popcountll(word);
            if (count > 0xFFFFFFFFull) {
                err = "compact layout holds at most 2^32-1 fluid nodes";
                return false;
            }
            while ((uint64_t)out.wstart.size() * 64 < count) out.wstart.push_back((uint32_t)(r * W + w));
        }
    }
    out.fluid = (int64_t)count;

    // slot of node x of row r, or kNoSlot when it is solid
    auto slot = [&](int64_t r, int x) -> uint32_t {
        const size_t k = (size_t)(r * W + (x >> 6));
        const uint64_t word = out.bits[k];
        if (!((word >> (x & 63)) & 1)) return kNoSlot;
        return out.base[k] + (uint32_t)__builtin_popcountll(word & ((1ull << (x & 63)) - 1ull));
    };
    const int64_t prow = (int64_t)(ny + 2) * (nz + 2);
    out.recs.assign((size_t)(prow * W), SegRec{0, 0, kNoSlot, kNoSlot, 0, 0});
    for (int zz = -1; zz <= nz; ++zz) {
        for (int yy = -1; yy <= ny; ++yy) {
            int y = yy, z = zz;
            bool inside = true;
            if (y < 0 || y >= ny) {
                if (per[1]) y = (y + ny) % ny;
                else inside = false;
            }
            if (z < 0 || z >= nz) {
                if (per[2]) z = (z + nz) % nz;
                else inside = false;
            }
            if (!inside) continue;  // behind a wall: an empty row (every node solid)
            const int64_t r = y + (int64_t)ny * z;
            for (int w = 0; w < W; ++w) {
                SegRec& s = out.recs[(size_t)(rec_row(yy, zz, ny) * W + w)];
                s.bits = out.bits[(size_t)(r * W + w)];
                s.base = out.base[(size_t)(r * W + w)];
                const int x0 = 64 * w, xl = std::min(x0 + 63, nx - 1);
                if (x0 > 0) s.lidx = slot(r, x0 - 1);
                else s.lidx = per[0] ? slot(r, nx - 1) : kNoSlot;
                if (xl + 1 < nx) s.ridx = slot(r, xl + 1);
                else s.ridx = per[0] ? slot(r, 0) : kNoSlot;
            }
        }
    }
    return true;
}

uint64_t payload_checksum(const void* data, size_t n)
{
    const uint64_t kBasis = 14695981039346656037ull, kPrime = 1099511628211ull;
    const unsigned char* p = (const unsigned char*)data;
    uint64_t h[4] = {kBasis, kBasis ^ 1, kBasis ^ 2, kBasis ^ 3};
    const size_t nw = n / 8;
    size_t i = 0;
    for (; i + 4 <= nw; i += 4) {
        for (int k = 0; k < 4; ++k) {
            uint64_t w;
            memcpy(&w, p + 8 * (i + k), 8);
            h[k] = (h[k] ^ w) * kPrime;
        }
    }
    for (; i < nw; ++i) {
        uint64_t w;
        memcpy(&w, p + 8 * i, 8);
        h[0] = (h[0] ^ w) * kPrime;
    }
    for (size_t b = 8 * nw; b < n; ++b) h[1] = (h[1] ^ p[b]) * kPrime;
    uint64_t r = kBasis;
    for (int k = 0; k < 4; ++k) r = (r ^ h[k]) * kPrime;
    return (r ^ (uint64_t)n) * kPrime;
}

uint64_t checkpoint_checksum(const CkptHeader& h, const void* payload, size_t n)
{
    CkptHeader z = h;
    z.checksum = 0;
    return (payload_checksum(&z, sizeof z) * 1099511628211ull) ^ payload_checksum(payload, n);
}

void checkpoint_sizes(const lbm_desc& d, bool has_tau, int64_t stride, CkptHeader& h)
{
    const int64_t N = (int64_t)d.nx * d.ny * d.nz;
    const int W = (d.nx + 63) / 64;
    h.pdf_bytes = (uint64_t)lattice_q(d.lattice) * (uint64_t)stride * prec_bytes(d.precision);
    h.tau_bytes = has_tau ? (uint64_t)stride * (d.precision == LBM_FP64 ? 8 : 4) : 0;
    h.mask_bytes = d.layout == LBM_DENSE ? (uint64_t)N : (uint64_t)W * d.ny * d.nz * 8;
    h.uprev_bytes = (uint64_t)3 * stride * sizeof(double);
}

namespace {
int bad(std::string& err, const char* msg)
{
    err = msg;
    return LBM_EFORMAT;
}
}  // namespace

int parse_checkpoint(const lbm_desc& d, bool has_tau, const void* blob, size_t bytes, CkptView& v,
                     std::string& err)
{
    CkptHeader& h = v.h;
    if (bytes < sizeof h) return bad(err, "checkpoint truncated (header)");
    memcpy(&h, blob, sizeof h);
    if (memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != kCkptVersion || h.header_bytes != sizeof h)
        return bad(err, "not a checkpoint of this library version");
    if (memcmp(&h.desc, &d, sizeof(lbm_desc)) != 0 || h.q != lattice_q(d.lattice))
        return bad(err, "checkpoint was saved from a different domain descriptor");
    const int64_t N = (int64_t)d.nx * d.ny * d.nz;
    if (h.t < 0) return bad(err, "checkpoint time is negative");
    if (h.parity != 0 && h.parity != 1) return bad(err, "checkpoint AA phase is not 0 or 1");
    if (d.scheme == LBM_AB && h.parity != 0) return bad(err, "checkpoint of an A/B domain with an AA phase");
    if (h.fluid < 0 || h.fluid > N) return bad(err, "checkpoint fluid count outside 0..N");
    const int64_t stride = d.layout == LBM_DENSE ? N : compact_stride(h.fluid, prec_bytes(d.precision));
    if (h.stride != stride) return bad(err, "checkpoint stride does not match its fluid count");
    CkptHeader want = h;
    checkpoint_sizes(d, has_tau, stride, want);
    if (h.pdf_bytes != want.pdf_bytes || h.tau_bytes != want.tau_bytes || h.mask_bytes != want.mask_bytes ||
        h.uprev_bytes != want.uprev_bytes)
        return bad(err, "checkpoint sizes do not match the domain");
    const uint64_t payload = h.pdf_bytes + h.tau_bytes + h.mask_bytes + h.uprev_bytes;
    if ((uint64_t)(bytes - sizeof h) < payload) return bad(err, "checkpoint truncated");
    const char* p = (const char*)blob + sizeof h;
    if (checkpoint_checksum(h, p, (size_t)payload) != h.checksum) return bad(err, "checkpoint checksum mismatch");
    v.pdf = p;
    v.tau = h.tau_bytes ? p + h.pdf_bytes : nullptr;
    v.mask = p + h.pdf_bytes + h.tau_bytes;
    v.uprev = v.mask + h.mask_bytes;
    int64_t fluid = 0;
    if (d.layout == LBM_DENSE) {
        for (int64_t n = 0; n < N; ++n) {
            const uint8_t m = (uint8_t)v.mask[n];
            if (m > 1) return bad(err, "checkpoint mask byte is neither 0 nor 1");
            fluid += m == 0;
        }
    } else {
        const int W = (d.nx + 63) / 64;
        const int tail = d.nx & 63;  // valid bits of a row's last word (0: all 64)
        const uint64_t past = tail ? ~((1ull << tail) - 1ull) : 0ull;
        const int64_t rows = (int64_t)d.ny * d.nz;
        for (int64_t r = 0; r < rows; ++r) {
            for (int w = 0; w < W; ++w) {
                uint64_t word;
                memcpy(&word, v.mask + 8 * (r * W + w), 8);
                if (w == W - 1 && (word & past)) return bad(err, "checkpoint bitmap marks a node past a row end");
                fluid += __builtin_popcountll(word);
            }
        }
    }
    if (fluid != h.fluid) return bad(err, "checkpoint mask does not hold the recorded fluid count");
    return LBM_OK;
}

void checkpoint_mask(const lbm_desc& d, const CkptView& v, std::vector<uint8_t>& mask)
{
    const int64_t N = (int64_t)d.nx * d.ny * d.nz;
    mask.assign((size_t)N, 1);
    if (d.layout == LBM_DENSE) {
        memcpy(mask.data(), v.mask, (size_t)N);
        return;
    }
    const int W = (d.nx + 63) / 64;
    const int64_t rows = (int64_t)d.ny * d.nz;
    for (int64_t r = 0; r < rows; ++r)
        for (int x = 0; x < d.nx; ++x) {
            uint64_t word;
            memcpy(&word, v.mask + 8 * (r * W + (x >> 6)), 8);
            mask[(size_t)(r * d.nx + x)] = ((word >> (x & 63)) & 1) ? 0 : 1;
        }
}

}  // namespace lbm
