// host_checks.cpp -- checks of the library's host-side logic (host.cpp),
// built with the address and undefined-behaviour sanitizers and run on the
// CPU by tests/test_sanitizers.py.  Covers: descriptor and rheology
// validation, the compact-layout builder against a direct computation from
// the mask, and checkpoint parsing (valid blobs, every truncation, single
// byte flips, and consistent-looking blobs with inconsistent contents).
// Prints "host checks: ok" and exits 0 when everything holds.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "host.hpp"

using namespace lbm;

static int failures = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

// xorshift64*: the checks' own seeded generator
static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t rnd()
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * 2685821657736338717ull;
}

static lbm_desc make_desc(int lat, int nx, int ny, int nz, const int per[3], int prec, int scheme, int layout)
{
    lbm_desc d;
    memset(&d, 0, sizeof d);
    d.lattice = lat;
    d.nx = nx;
    d.ny = ny;
    d.nz = nz;
    for (int k = 0; k < 3; ++k) d.periodic[k] = per[k];
    d.precision = prec;
    d.scheme = scheme;
    d.layout = layout;
    return d;
}

static lbm_rheology make_rh(int op)
{
    lbm_rheology r;
    memset(&r, 0, sizeof r);
    r.op = op;
    r.nu_p = 0.1;
    r.sigma_y = 1e-4;
    r.rho0 = 1.0;
    r.m = 1e4;
    r.gamma_c = 1e-8;
    r.lambda_trt = 0.25;
    r.fp16_scale_log2 = 14;
    r.hb_n = 1.0;
    return r;
}

static void check_validation()
{
    std::string err;
    const int per[3] = {1, 0, 1};
    lbm_desc d = make_desc(2, 8, 8, 8, per, LBM_FP64, LBM_AA, LBM_COMPACT);
    CHECK(validate_desc(&d, err) == LBM_OK);
    CHECK(validate_desc(nullptr, err) == LBM_EINVAL);
    lbm_desc b = d;
    b.lattice = 7;
    CHECK(validate_desc(&b, err) == LBM_EINVAL);
    b = d;
    b.nx = 0;
    CHECK(validate_desc(&b, err) == LBM_EINVAL);
    b = d;
    b.lattice = LBM_D2Q9;
    CHECK(validate_desc(&b, err) == LBM_EINVAL);  // nz != 1
    b = d;
    b.nx = b.ny = b.nz = 1 << 13;
    CHECK(validate_desc(&b, err) == LBM_EINVAL);  // too large
    b = d;
    b.precision = 3;
    CHECK(validate_desc(&b, err) == LBM_EINVAL);
    b = d;
    b.scheme = -1;
    CHECK(validate_desc(&b, err) == LBM_EINVAL);
    b = d;
    b.layout = 2;
    CHECK(validate_desc(&b, err) == LBM_EINVAL);

    for (int op = 0; op < 4; ++op) {
        lbm_rheology r = make_rh(op);
        CHECK(validate_rheology(&r, err) == LBM_OK);
        lbm_rheology x = r;
        x.nu_p = 0;
        CHECK(validate_rheology(&x, err) == LBM_EINVAL);
        x = r;
        x.sigma_y = NAN;
        CHECK(validate_rheology(&x, err) == LBM_EINVAL);
        x = r;
        x.g[1] = INFINITY;
        CHECK(validate_rheology(&x, err) == LBM_EINVAL);
        x = r;
        x.fp16_scale_log2 = 25;
        CHECK(validate_rheology(&x, err) == LBM_EINVAL);
        x = r;
        x.fallback_band = -1;
        CHECK(validate_rheology(&x, err) == LBM_EINVAL);
        x = r;
        x.flow_axis = 4;
        CHECK(validate_rheology(&x, err) == LBM_EINVAL);
        x = r;
        x.mrt_even = 2.0;
        CHECK(validate_rheology(&x, err) == LBM_EINVAL);
    }
    lbm_rheology r = make_rh(LBM_PR);
    r.gamma_c = 0;
    CHECK(validate_rheology(&r, err) == LBM_EINVAL);
    r = make_rh(LBM_IRHB);
    r.hb_n = 0.1;
    CHECK(validate_rheology(&r, err) == LBM_EINVAL);
    r = make_rh(LBM_IR);
    r.mrt_bulk = 1.2;
    CHECK(validate_rheology(&r, err) == LBM_EINVAL);
    r = make_rh(7);
    CHECK(validate_rheology(&r, err) == LBM_EINVAL);
    CHECK(validate_rheology(nullptr, err) == LBM_EINVAL);
}

// slot of (x, y, z) computed straight from the mask, or kNoSlot
static uint32_t direct_slot(const std::vector<uint8_t>& m, int nx, int ny, int x, int y, int z)
{
    const int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
    if (m[(size_t)n]) return kNoSlot;
    uint32_t k = 0;
    for (int64_t j = 0; j < n; ++j) k += m[(size_t)j] == 0;
    return k;
}

static void check_builder(int nx, int ny, int nz, const int per[3], double solid_fraction)
{
    const int64_t N = (int64_t)nx * ny * nz;
    std::vector<uint8_t> m((size_t)N);
    for (auto& v : m) v = (double)(rnd() >> 11) * (1.0 / 9007199254740992.0) < solid_fraction ? 1 : 0;
    CompactMask cm;
    std::string err;
    CHECK(build_compact_mask(nx, ny, nz, per, m.data(), cm, err));
    const int W = (nx + 63) / 64;
    CHECK(cm.W == W);
    int64_t fluid = 0;
    for (auto v : m) fluid += v == 0;
    CHECK(cm.fluid == fluid);
    CHECK(cm.bits.size() == (size_t)(W * ny * nz) && cm.base.size() == cm.bits.size());
    CHECK(cm.wstart.size() == (size_t)((fluid + 63) / 64));
    CHECK(cm.recs.size() == (size_t)W * (ny + 2) * (nz + 2));
    // bitmap and bases
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int w = 0; w < W; ++w) {
                const size_t k = (size_t)((y + (int64_t)ny * z) * W + w);
                for (int b = 0; b < 64; ++b) {
                    const int x = 64 * w + b;
                    const bool fl = x < nx && m[(size_t)(x + (int64_t)nx * (y + (int64_t)ny * z))] == 0;
                    CHECK((((cm.bits[k] >> b) & 1) != 0) == fl);
                    if (fl)
                        CHECK(cm.base[k] + (uint32_t)__builtin_popcountll(cm.bits[k] & ((1ull << b) - 1ull)) ==
                              direct_slot(m, nx, ny, x, y, z));
                }
            }
    // group table: word holding slot 64 g
    for (size_t g = 0; g < cm.wstart.size(); ++g) {
        const uint32_t w = cm.wstart[g];
        CHECK(w < cm.bits.size());
        if (w >= cm.bits.size()) continue;
        const uint64_t s = 64 * (uint64_t)g;
        CHECK(cm.base[w] <= s && s < cm.base[w] + (uint64_t)__builtin_popcountll(cm.bits[w]));
    }
    // segment records with halo rows
    for (int zz = -1; zz <= nz; ++zz)
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
            for (int w = 0; w < W; ++w) {
                const SegRec& r = cm.recs[(size_t)(rec_row(yy, zz, ny) * W + w)];
                if (!inside) {
                    CHECK(r.bits == 0 && r.lidx == kNoSlot && r.ridx == kNoSlot);
                    continue;
                }
                const size_t k = (size_t)((y + (int64_t)ny * z) * W + w);
                CHECK(r.bits == cm.bits[k] && r.base == cm.base[k]);
                const int x0 = 64 * w, xl = x0 + 63 < nx - 1 ? x0 + 63 : nx - 1;
                uint32_t want_l = kNoSlot, want_r = kNoSlot;
                if (x0 > 0) want_l = direct_slot(m, nx, ny, x0 - 1, y, z);
                else if (per[0]) want_l = direct_slot(m, nx, ny, nx - 1, y, z);
                if (xl + 1 < nx) want_r = direct_slot(m, nx, ny, xl + 1, y, z);
                else if (per[0]) want_r = direct_slot(m, nx, ny, 0, y, z);
                CHECK(r.lidx == want_l && r.ridx == want_r);
            }
        }
}

// A checkpoint blob for desc with the given mask and random payload values.
static std::vector<char> make_blob(const lbm_desc& d, bool has_tau, const std::vector<uint8_t>& m, int64_t t,
                                   int parity)
{
    const int per[3] = {d.periodic[0], d.periodic[1], d.lattice == LBM_D2Q9 ? 1 : d.periodic[2]};
    CompactMask cm;
    std::string err;
    build_compact_mask(d.nx, d.ny, d.nz, per, m.data(), cm, err);
    const int64_t N = (int64_t)d.nx * d.ny * d.nz;
    CkptHeader h;
    memset(&h, 0, sizeof h);
    memcpy(h.magic, kCkptMagic, 8);
    h.version = kCkptVersion;
    h.header_bytes = sizeof h;
    h.desc = d;
    h.rh = make_rh(has_tau ? LBM_PR : LBM_IR);
    h.t = t;
    h.fluid = cm.fluid;
    h.stride = d.layout == LBM_DENSE ? N : compact_stride(cm.fluid, prec_bytes(d.precision));
    h.parity = parity;
    h.q = lattice_q(d.lattice);
    checkpoint_sizes(d, has_tau, h.stride, h);
    const size_t payload = h.pdf_bytes + h.tau_bytes + h.mask_bytes + h.uprev_bytes;
    std::vector<char> blob(sizeof h + payload);
    char* p = blob.data() + sizeof h;
    for (size_t k = 0; k < h.pdf_bytes + h.tau_bytes; ++k) p[k] = (char)rnd();
    char* mk = p + h.pdf_bytes + h.tau_bytes;
    if (d.layout == LBM_DENSE) memcpy(mk, m.data(), (size_t)N);
    else memcpy(mk, cm.bits.data(), h.mask_bytes);
    for (size_t k = 0; k < h.uprev_bytes; ++k) mk[h.mask_bytes + k] = (char)rnd();
    h.checksum = checkpoint_checksum(h, p, payload);
    memcpy(blob.data(), &h, sizeof h);
    return blob;
}

// parse from an exactly-sized heap copy (so a read past the end is caught)
static int parse_exact(const lbm_desc& d, bool has_tau, const std::vector<char>& blob, size_t bytes)
{
    char* buf = (char*)malloc(bytes ? bytes : 1);
    memcpy(buf, blob.data(), bytes);
    CkptView v;
    std::string err;
    const int rc = parse_checkpoint(d, has_tau, buf, bytes, v, err);
    if (rc == LBM_OK) {
        std::vector<uint8_t> back;
        checkpoint_mask(d, v, back);
    }
    free(buf);
    return rc;
}

// re-seal a modified blob with a correct checksum
static void reseal(std::vector<char>& blob)
{
    CkptHeader h;
    memcpy(&h, blob.data(), sizeof h);
    h.checksum = checkpoint_checksum(h, blob.data() + sizeof h, blob.size() - sizeof h);
    memcpy(blob.data(), &h, sizeof h);
}

static void check_checkpoints(int layout, int scheme, bool has_tau)
{
    const int per[3] = {1, 0, 1};
    const lbm_desc d = make_desc(2, 70, 5, 3, per, LBM_FP32, scheme, layout);
    const int64_t N = (int64_t)d.nx * d.ny * d.nz;
    std::vector<uint8_t> m((size_t)N);
    for (auto& v : m) v = (rnd() & 3) == 0 ? 1 : 0;
    const int parity = scheme == LBM_AA ? 1 : 0;
    const std::vector<char> good = make_blob(d, has_tau, m, 123, parity);
    CHECK(parse_exact(d, has_tau, good, good.size()) == LBM_OK);
    // the mask read back is the one saved
    {
        CkptView v;
        std::string err;
        CHECK(parse_checkpoint(d, has_tau, good.data(), good.size(), v, err) == LBM_OK);
        std::vector<uint8_t> back;
        checkpoint_mask(d, v, back);
        CHECK(back == m);
    }
    // another descriptor or operator family
    lbm_desc d2 = d;
    d2.ny = 6;
    CHECK(parse_exact(d2, has_tau, good, good.size()) == LBM_EFORMAT);
    CHECK(parse_exact(d, !has_tau, good, good.size()) == LBM_EFORMAT);
    // every truncation
    for (size_t b = 0; b < good.size(); b += (b < 512 ? 1 : 97)) CHECK(parse_exact(d, has_tau, good, b) == LBM_EFORMAT);
    // single byte flips anywhere
    for (int k = 0; k < 400; ++k) {
        std::vector<char> bad = good;
        const size_t at = (size_t)(rnd() % bad.size());
        bad[at] ^= (char)(1 + rnd() % 255);
        CHECK(parse_exact(d, has_tau, bad, bad.size()) == LBM_EFORMAT);
    }
    // consistent-looking (re-sealed) blobs with inconsistent contents
    auto with_header = [&](void (*edit)(CkptHeader&)) {
        std::vector<char> bad = good;
        CkptHeader h;
        memcpy(&h, bad.data(), sizeof h);
        edit(h);
        memcpy(bad.data(), &h, sizeof h);
        reseal(bad);
        return parse_exact(d, has_tau, bad, bad.size());
    };
    CHECK(with_header([](CkptHeader& h) { h.t = -1; }) == LBM_EFORMAT);
    CHECK(with_header([](CkptHeader& h) { h.parity = 2; }) == LBM_EFORMAT);
    CHECK(with_header([](CkptHeader& h) { h.fluid += 1; }) == LBM_EFORMAT);
    CHECK(with_header([](CkptHeader& h) { h.stride += 64; }) == LBM_EFORMAT);
    CHECK(with_header([](CkptHeader& h) { h.q = 19; }) == LBM_EFORMAT);
    CHECK(with_header([](CkptHeader& h) { h.version = 2; }) == LBM_EFORMAT);
    CHECK(with_header([](CkptHeader& h) { h.pdf_bytes += 4; }) == LBM_EFORMAT);
    if (scheme == LBM_AB) CHECK(with_header([](CkptHeader& h) { h.parity = 1; }) == LBM_EFORMAT);
    // the informational rheology may differ (a state continued under other parameters)
    CHECK(with_header([](CkptHeader& h) { h.rh.m = 1e9; }) == LBM_OK);
    CkptHeader h;
    memcpy(&h, good.data(), sizeof h);
    char* mk = (char*)nullptr;
    {
        std::vector<char> bad = good;
        mk = bad.data() + sizeof h + h.pdf_bytes + h.tau_bytes;
        if (layout == LBM_DENSE) {
            mk[5] = 2;  // neither 0 nor 1
        } else {
            uint64_t w;
            const int W = (d.nx + 63) / 64;
            memcpy(&w, mk + 8 * (W - 1), 8);
            w |= 1ull << 63;  // a fluid bit past the row end (nx = 70)
            memcpy(mk + 8 * (W - 1), &w, 8);
        }
        reseal(bad);
        CHECK(parse_exact(d, has_tau, bad, bad.size()) == LBM_EFORMAT);
    }
    {
        // one mask bit or byte flipped: the fluid count no longer matches
        std::vector<char> bad = good;
        mk = bad.data() + sizeof h + h.pdf_bytes + h.tau_bytes;
        if (layout == LBM_DENSE) mk[7] ^= 1;
        else mk[0] ^= 1;
        reseal(bad);
        CHECK(parse_exact(d, has_tau, bad, bad.size()) == LBM_EFORMAT);
    }
}

int main()
{
    check_validation();
    const int pers[4][3] = {{1, 1, 1}, {0, 0, 0}, {1, 0, 1}, {0, 1, 0}};
    const int dims[][3] = {{1, 1, 1}, {1, 3, 2}, {63, 2, 2}, {64, 3, 1}, {65, 2, 3}, {130, 3, 2}, {200, 1, 1}};
    for (const auto& dm : dims)
        for (const auto& pr : pers)
            for (double f : {0.0, 0.3, 0.85, 1.0}) check_builder(dm[0], dm[1], dm[2], pr, f);
    std::string err;
    CompactMask cm;
    const int per2[3] = {1, 1, 1};
    CHECK(build_compact_mask(3, 2, 1, per2, nullptr, cm, err) && cm.fluid == 6);
    CHECK(compact_stride(0, 8) >= 64);
    for (int64_t nf : {0LL, 1LL, 63LL, 64LL, 65LL, 4096LL, 11743335LL}) {
        for (size_t eb : {2, 4, 8}) {
            const int64_t S = compact_stride(nf, eb);
            const int64_t P = 65536 / (int64_t)eb;
            CHECK(S >= nf && S % 64 == 0 && S - (nf + 63) / 64 * 64 < P);
            CHECK(S % P >= P / 4 && S % P < 3 * P / 4);
        }
    }
    for (int layout : {LBM_COMPACT, LBM_DENSE})
        for (int scheme : {LBM_AA, LBM_AB})
            for (bool tau : {true, false}) check_checkpoints(layout, scheme, tau);
    if (failures) {
        fprintf(stderr, "host checks: %d failures\n", failures);
        return 1;
    }
    printf("host checks: ok\n");
    return 0;
}
