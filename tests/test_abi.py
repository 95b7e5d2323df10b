"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/lbm.h declares, its velocity sets are the
oracle's (as sets, with the same weights and opposites), and descriptor and
rheology validation reject bad input before any device work."""
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
