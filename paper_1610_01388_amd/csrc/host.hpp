// host.hpp -- host-side logic of the library that touches no device:
// the compact-layout builder (bitmap, word bases, group table, segment
// records), the population stride, and the checkpoint format with its
// validation.  Plain C++ (no HIP), so that it also builds and runs under the
// address and undefined-behaviour sanitizers on a machine without a GPU.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "layout.hpp"
#include "lbm.h"

namespace lbm {

// Velocity count of a lattice code (-1 if unknown).
inline int lattice_q(int lat) { return lat == 0 ? 9 : lat == 1 ? 19 : lat == 2 ? 27 : -1; }
inline int lattice_d(int lat) { return lat == 0 ? 2 : 3; }
inline size_t prec_bytes(int p) { return p == LBM_FP64 ? 8 : p == LBM_FP32 ? 4 : 2; }

// Validation of a descriptor and a rheology (the rules lbm_create states):
// LBM_OK, or LBM_EINVAL with a message.
int validate_desc(const lbm_desc* d, std::string& err);
int validate_rheology(const lbm_rheology* r, std::string& err);

// Direction stride of the compact layout's population arrays for nf fluid
// nodes of elem_bytes each: nf rounded up to 64, then padded (by less than
// 64 KiB) until its byte size modulo 64 KiB lies in the middle half of that
// period, so that the Q arrays of one node do not all start on the same HBM
// channels.
int64_t compact_stride(int64_t nf, size_t elem_bytes);

// Compact layout of one solid mask (W = ceil(nx / 64) words per row).
struct CompactMask {
    int W = 0;
    std::vector<uint64_t> bits;    // [row][W], row = y + ny z; bit set = fluid
    std::vector<uint32_t> base;    // [row][W]: slot of the first fluid node at or after x = 64 w
    std::vector<uint32_t> wstart;  // per group of 64 slots: the word [row][W] holding its first slot
    std::vector<SegRec> recs;      // [(ny + 2)(nz + 2)][W], see SegRec
    int64_t fluid = 0;
};

// Build the compact layout of mask (N = nx ny nz bytes, nonzero = solid; NULL
// = all fluid) for the periodic flags per (nonzero = periodic).  Returns
// false with a message when the fluid count exceeds 2^32 - 1.
bool build_compact_mask(int nx, int ny, int nz, const int per[3], const uint8_t* mask, CompactMask& out,
                        std::string& err);

// Checksum of a byte range: FNV-1a over 64-bit little-endian words in four
// interleaved lanes (then the tail bytes), the lanes combined at the end.
uint64_t payload_checksum(const void* data, size_t n);

// Checkpoint blob: this header, then the payload -- the raw population
// storage (pdf_bytes), the PR relaxation-time field (tau_bytes), the mask
// (mask_bytes: the dense layout's N mask bytes, 1 = solid, or the compact
// layout's fluid bitmap, ny nz rows of W 64-bit words) and the residual
// monitor's reference velocity (uprev_bytes, 3 x stride doubles).
struct CkptHeader {
    char magic[8];
    uint32_t version, header_bytes;
    lbm_desc desc;
    lbm_rheology rh;
    int64_t t, stride, fluid;
    int32_t parity, q;
    uint64_t pdf_bytes, tau_bytes, mask_bytes, uprev_bytes;
    uint64_t checksum;  // checkpoint_checksum of the header (this field zero) and the payload
};
static_assert(sizeof(CkptHeader) == 248, "the checkpoint header has no padding bytes");
constexpr uint32_t kCkptVersion = 3;
extern const char kCkptMagic[8];

// Checksum of a checkpoint: of its header with the checksum field zero and of
// its payload, combined, so that a change anywhere in the blob changes it.
uint64_t checkpoint_checksum(const CkptHeader& h, const void* payload, size_t n);

// Byte sizes of the payload parts for a domain (desc, keeps a relaxation-time
// field or not) holding `fluid` fluid nodes at direction stride `stride`.
void checkpoint_sizes(const lbm_desc& d, bool has_tau, int64_t stride, CkptHeader& h);

// A validated checkpoint: its header and the payload parts.
struct CkptView {
    CkptHeader h;
    const char* pdf = nullptr;
    const char* tau = nullptr;
    const char* mask = nullptr;
    const char* uprev = nullptr;
};

// Validate a checkpoint blob against a domain (descriptor d; has_tau: it
// keeps a relaxation-time field) on the host, before any device work:
// header, descriptor, sizes, checksum, time >= 0, AA phase in {0, 1}
// (0 for A/B), and a mask consistent with the header -- dense: bytes in
// {0, 1} with `fluid` zeros; compact: no fluid bit past a row's end and
// `fluid` bits set -- and a stride equal to the one the layout derives from
// the fluid count.  Returns LBM_OK, or LBM_EFORMAT with a message.
int parse_checkpoint(const lbm_desc& d, bool has_tau, const void* blob, size_t bytes, CkptView& v,
                     std::string& err);

// The solid mask (N bytes, 1 = solid) of a validated checkpoint.
void checkpoint_mask(const lbm_desc& d, const CkptView& v, std::vector<uint8_t>& mask);

}  // namespace lbm
