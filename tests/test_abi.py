"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/lbm.h declares, its velocity sets are the
oracle's (as sets, with the same weights and opposites), and descriptor and
rheology validation reject bad input before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1610_01388_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_\w+)\s*\(", src)))


def test_exports_every_declared_function():
    L = lbm.load_library()
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert sorted(lbm.EXPORTS) == names


@pytest.mark.parametrize("lat", [0, 1, 2])
def test_velocity_sets_match_oracle(lat):
    c, w, opp = lbm.lbm_lattice_info(lat)
    _, co, wo, _ = oracle.lattice_info(lat)
    assert {tuple(v) for v in c} == {tuple(v) for v in co}
    for k, v in enumerate(c):
        i = int(np.flatnonzero((co == v).all(1))[0])
        assert w[k] == wo[i]
        assert np.array_equal(c[opp[k]], -v)
    assert tuple(c[0]) == (0, 0, 0)


def _desc(**kw):
    d = dict(lattice="D3Q19", dims=(8, 8, 8), periodic=(1, 1, 1), precision="FP64", scheme="AA",
             layout="COMPACT")
    d.update(kw)
    return lbm.make_desc(d["lattice"], d["dims"], d["periodic"], d["precision"], d["scheme"], d["layout"])


@pytest.mark.parametrize("kw,rkw", [
    (dict(dims=(0, 8, 8)), {}),
    (dict(lattice=5), {}),
    (dict(lattice="D2Q9", dims=(8, 8, 2)), {}),
    (dict(precision=7), {}),
    (dict(scheme=3), {}),
    (dict(layout=4), {}),
    ({}, dict(nu_p=0.0)),
    ({}, dict(nu_p=-0.1)),
    ({}, dict(sigma_y=-1e-5)),
    ({}, dict(rho0=0.0)),
    ({}, dict(op="PR", m=-1.0)),
    ({}, dict(op="PR", gamma_c=0.0)),
    ({}, dict(op="PR", lambda_trt=0.0)),
    ({}, dict(fp16_scale_log2=30)),
    ({}, dict(flow_axis=4)),
    ({}, dict(op="PR", mrt_bulk=2.5)),
    ({}, dict(op="PR", mrt_even=-0.1)),
    ({}, dict(op="IR", mrt_even=1.2)),
    ({}, dict(op="PRI", mrt_bulk=1.2)),
    ({}, dict(flow_axis=-1)),
    ({}, dict(fallback_band=-1.0)),
])
def test_create_rejects_invalid(kw, rkw):
    r = dict(op="IR", nu_p=0.1)
    r.update(rkw)
    op, nu = r.pop("op"), r.pop("nu_p")
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(_desc(**kw), lbm.make_rheology(op, nu, **r))
    assert e.value.code == -1


def test_query_sizes():
    d = _desc(lattice="D3Q27", dims=(10, 12, 14), precision="FP32", scheme="AB")
    s = lbm.lbm_query_sizes(d, lbm.make_rheology("PR", 0.1, 1e-5, 1e4))
    N = 10 * 12 * 14
    assert s.pdf_bytes >= 2 * 27 * N * 4 and s.pdf_bytes % 256 == 0
    assert s.tau_bytes >= N * 4
    assert s.mask_bytes >= N
    s2 = lbm.lbm_query_sizes(_desc(lattice="D3Q27", dims=(10, 12, 14), precision="FP16"),
                             lbm.make_rheology("IR", 0.1))
    assert s2.tau_bytes == 0 and s2.pdf_bytes >= 27 * N * 2


def test_unbound_domain_refuses_work():
    h = lbm.lbm_create(_desc(layout="DENSE"), lbm.make_rheology("IR", 0.1))
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_step(h, 1)
    assert e.value.code == -4
    with pytest.raises(lbm.LbmError):
        lbm.lbm_set_tile(h, 64, 64, 1)
    lbm.lbm_set_tile(h, 8, 8, 2)
    assert lbm.lbm_get_tile(h) == (8, 8, 2)
    lbm.lbm_destroy(h)
    h = lbm.lbm_create(_desc(layout="COMPACT"), lbm.make_rheology("IR", 0.1))
    with pytest.raises(lbm.LbmError):
        lbm.lbm_set_tile(h, 8, 8, 2)  # compact needs one wavefront per 64-node row segment
    lbm.lbm_set_tile(h, 64, 2, 2)
    lbm.lbm_set_tile(h, 128, 2, 1)  # two adjacent row segments per block
    lbm.lbm_set_tile(h, 256, 1, 1)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_set_tile(h, 192, 1, 1)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_set_pull_form(h, 3)
    assert e.value.code == -1
    for form in ("SLOTS", "ROWS"):
        lbm.lbm_set_pull_form(h, form)
        assert lbm.lbm_get_pull_form(h) == form
    lbm.lbm_destroy(h)


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the ABI structs have the header's size and field
    offsets (compiled with the host C compiler against include/lbm.h)."""
    import ctypes
    import subprocess
    structs = {"lbm_desc": lbm.lbm_desc, "lbm_rheology": lbm.lbm_rheology, "lbm_monitor": lbm.lbm_monitor,
               "lbm_sizes": lbm.lbm_sizes}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines.append("return 0; }")
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l)}
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f in cls._fields_:
            assert got[(name, f[0])] == getattr(cls, f[0]).offset, (name, f[0])


def test_implicit_pr_needs_no_tau_and_batches_reject_it():
    d = _desc(lattice="D3Q19", dims=(8, 9, 10))
    s = lbm.lbm_query_sizes(d, lbm.make_rheology("PRI", 0.1, 1e-4, 1e4))
    assert s.tau_bytes == 0
    assert lbm.lbm_query_sizes(d, lbm.make_rheology("PR", 0.1, 1e-4, 1e4)).tau_bytes > 0
    h = lbm.lbm_create(d, lbm.make_rheology("PRI", 0.1, 1e-4, 1e4))
    lbm.lbm_destroy(h)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_batch_query_sizes([lbm.make_desc("D3Q19", (8, 8, 4), (0, 0, 1), "FP32", "AA")],
                                  [lbm.make_rheology("PRI", 0.1, 1e-4, 1e4)])
    assert e.value.code == -1


def test_irhb_validation_and_batches_reject_it():
    for n in (0.1, 6.0):
        with pytest.raises(lbm.LbmError):
            lbm.lbm_create(_desc(), lbm.make_rheology("IRHB", 0.01, 1e-4, hb_n=n))
    with pytest.raises(lbm.LbmError):
        lbm.lbm_create(_desc(), lbm.make_rheology("IRHB", 0.01, 1e-4, hb_n=0.5, mrt_even=1.2))
    h = lbm.lbm_create(_desc(), lbm.make_rheology("IRHB", 0.01, 1e-4, hb_n=0.5))
    lbm.lbm_destroy(h)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_batch_query_sizes([lbm.make_desc("D3Q19", (8, 8, 4), (0, 0, 1), "FP32", "AA")],
                                  [lbm.make_rheology("IRHB", 0.01, 1e-4, hb_n=0.5)])
    assert e.value.code == -1


def test_batches_reject_mrt():
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_batch_query_sizes([lbm.make_desc("D3Q19", (8, 8, 4), (0, 0, 1), "FP32", "AA")],
                                  [lbm.make_rheology("PR", 0.1, 1e-4, 1e4, mrt_even=1.5)])
    assert e.value.code == -1


# --- checkpoint validation on the host (lbm_check_checkpoint) ----------------

class _CkptHeader(ctypes.Structure):
    _fields_ = [("magic", ctypes.c_char * 8), ("version", ctypes.c_uint32), ("header_bytes", ctypes.c_uint32),
                ("desc", lbm.lbm_desc), ("rh", lbm.lbm_rheology), ("t", ctypes.c_int64), ("stride", ctypes.c_int64),
                ("fluid", ctypes.c_int64), ("parity", ctypes.c_int32), ("q", ctypes.c_int32),
                ("pdf_bytes", ctypes.c_uint64), ("tau_bytes", ctypes.c_uint64), ("mask_bytes", ctypes.c_uint64),
                ("uprev_bytes", ctypes.c_uint64), ("checksum", ctypes.c_uint64)]


_P64, _B64, _M64 = 1099511628211, 14695981039346656037, (1 << 64) - 1


def _words_checksum(b: bytes) -> int:
    """The documented checksum: FNV-1a over 64-bit little-endian words in four
    interleaved lanes, a leftover word into lane 0, tail bytes into lane 1,
    the lanes combined, then the length."""
    h = [_B64, _B64 ^ 1, _B64 ^ 2, _B64 ^ 3]
    nw = len(b) // 8
    w = np.frombuffer(b[:8 * nw], dtype="<u8")
    full = nw - nw % 4
    for k in range(4):
        for v in w[k:full:4].tolist():
            h[k] = ((h[k] ^ v) * _P64) & _M64
    for v in w[full:].tolist():
        h[0] = ((h[0] ^ v) * _P64) & _M64
    for v in b[8 * nw:]:
        h[1] = ((h[1] ^ v) * _P64) & _M64
    r = _B64
    for k in range(4):
        r = ((r ^ h[k]) * _P64) & _M64
    return ((r ^ len(b)) * _P64) & _M64


def _blob(desc, rh, mask, t=5, parity=1, edit=None):
    """A checkpoint for (desc, rh) with the given solid mask, built from the
    format lbm.h documents; edit(header, payload) may change it before the
    checksum is taken."""
    N = desc.nx * desc.ny * desc.nz
    q = {0: 9, 1: 19, 2: 27}[desc.lattice]
    eb = {0: 8, 1: 4, 2: 2}[desc.precision]
    nf = int((mask == 0).sum())
    if desc.layout == 1:
        stride = N
        mbytes = mask.astype(np.uint8).tobytes()
    else:
        S, P = max(64, (nf + 63) // 64 * 64), 65536 // eb
        r = S % P
        stride = S if P // 4 <= r < 3 * P // 4 else S + ((P // 4 - r) % P + P) % P
        W = (desc.nx + 63) // 64
        words = np.zeros((desc.ny * desc.nz, W), dtype="<u8")
        fl = (mask.reshape(desc.ny * desc.nz, desc.nx) == 0)
        for x in range(desc.nx):
            words[:, x // 64] |= fl[:, x].astype(np.uint64) << np.uint64(x % 64)
        mbytes = words.tobytes()
    h = _CkptHeader()
    h.magic = b"LBMCKPT1"
    h.version, h.header_bytes = 3, ctypes.sizeof(_CkptHeader)
    h.desc, h.rh = desc, rh
    h.t, h.stride, h.fluid, h.parity, h.q = t, stride, nf, parity, q
    h.pdf_bytes = q * stride * eb
    h.tau_bytes = stride * (8 if desc.precision == 0 else 4) if rh.op == 0 else 0
    h.mask_bytes = len(mbytes)
    h.uprev_bytes = 3 * stride * 8
    rnd = np.random.default_rng(7)
    payload = bytearray(rnd.bytes(h.pdf_bytes + h.tau_bytes) + mbytes + rnd.bytes(h.uprev_bytes))
    if edit:
        edit(h, payload)
    h.checksum = 0
    hsum = _words_checksum(bytes(h))
    h.checksum = ((hsum * _P64) & _M64) ^ _words_checksum(bytes(payload))
    return bytes(h) + bytes(payload)


@pytest.mark.parametrize("layout", ["COMPACT", "DENSE"])
@pytest.mark.parametrize("op", ["PR", "IR"])
def test_check_checkpoint_on_the_host(layout, op):
    assert ctypes.sizeof(_CkptHeader) == 248
    desc = _desc(lattice="D3Q19", dims=(70, 5, 3), periodic=(1, 0, 1), precision="FP32", layout=layout)
    rh = lbm.make_rheology(op, 0.1, 1e-4, m=1e4)
    N = 70 * 5 * 3
    mask = (np.arange(N) % 7 == 0).astype(np.uint8)
    good = _blob(desc, rh, mask)
    lbm.lbm_check_checkpoint(desc, rh, good)  # accepted

    def rejected(blob, d=desc, r=rh):
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_check_checkpoint(d, r, blob)
        assert e.value.code == -6

    rejected(good[:-1])
    rejected(good[:100])
    flipped = bytearray(good)
    flipped[len(good) // 2] ^= 0x10
    rejected(bytes(flipped))
    rejected(good, d=_desc(lattice="D3Q19", dims=(70, 6, 3), periodic=(1, 0, 1), precision="FP32", layout=layout))
    rejected(good, r=lbm.make_rheology("IR" if op == "PR" else "PR", 0.1, 1e-4, m=1e4))  # tau field present/absent
    # consistent-looking (correct checksum) but inconsistent contents

    def set_header(**kw):
        def edit(h, payload):
            for k, v in kw.items():
                setattr(h, k, v)
        return edit

    rejected(_blob(desc, rh, mask, edit=set_header(t=-1)))
    rejected(_blob(desc, rh, mask, edit=set_header(parity=2)))
    rejected(_blob(desc, rh, mask, edit=set_header(fluid=int((mask == 0).sum()) + 1)))

    def mask_edit(h, payload):
        off = h.pdf_bytes + h.tau_bytes
        if layout == "DENSE":
            payload[off + 3] = 2  # neither 0 nor 1
        else:
            payload[off + 15] |= 0x80  # bit 63 of word 1 of row 0: x = 127, past the row end (nx = 70)
    rejected(_blob(desc, rh, mask, edit=mask_edit))
    # another rheology in the header is accepted (a state may be continued under other parameters)
    lbm.lbm_check_checkpoint(desc, rh, _blob(desc, rh, mask, edit=set_header(t=9)))
