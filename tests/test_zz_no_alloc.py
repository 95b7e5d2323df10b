"""The allocation-free monitor entry point (lbm_monitors_async) against the
on-demand monitors of lbm_monitors, through the C ABI: two calls in a row on
two domains, the second smaller.  The first domain has more nodes than 2048
blocks of 256, so its reduction walks the nodes with a grid stride.

Bars: counts and maxima (fluid, unyielded, nonfinite, umax, du_max) exactly
equal; sums (flux, mass, residual) within 1e-12 relative -- the two
reductions add the same per-node FP64 terms in different orders."""
import ctypes

import numpy as np
import pytest

from support import perm_lib_from_oracle, random_mask, random_state

pytestmark = pytest.mark.gpu


def _record(torch, lbm, dom):
    rec = torch.zeros(12, dtype=torch.float64, device=dom.device)
    lbm.lbm_monitors_async(dom.h, rec.data_ptr())
    dom.synchronize()
    raw = rec.cpu().numpy().tobytes()
    return lbm.lbm_monitor.from_buffer_copy(raw).as_dict()


def _case(lbm, dims, seed):
    lat = 2
    N = int(np.prod(dims))
    mask = random_mask(N, seed, 0.2)
    dom = lbm.Domain("D3Q27", dims, (1, 0, 1), "IR", 0.1, 5e-4, g=(2e-5, -1e-5, 5e-6))
    dom.set_mask(mask)
    P0, _ = random_state(lat, N, seed)
    dom.write_populations((P0 * (1 - mask)[None, :])[perm_lib_from_oracle(lat)])
    dom.set_monitor_interval(3)
    dom.step(7)  # fused records at 0, 3, 6 set the residual's reference velocity
    dom.history()
    return dom


def _same(a, b):
    for key in ("fluid", "unyielded", "nonfinite", "step", "fallback"):
        assert a[key] == b[key], key
    assert a["umax"] == b["umax"] and a["du_max"] == b["du_max"]
    assert np.max(np.abs(a["flux"] - b["flux"])) <= 1e-12 * np.max(np.abs(b["flux"]))
    assert abs(a["mass"] - b["mass"]) <= 1e-12 * b["mass"]
    assert abs(a["residual"] - b["residual"]) <= 1e-12 * b["residual"]


def test_monitors_async_matches_monitors_twice():
    import torch

    from paper_1610_01388_amd import lbm
    big = _case(lbm, (96, 80, 80), 31)  # 614 400 nodes > 2048 x 256
    assert big.N > 2048 * 256
    got = _record(torch, lbm, big)
    want = big.monitors()
    assert want["status"] == 0 and got["residual"] > 0
    _same(got, want)
    big.close()
    small = _case(lbm, (37, 11, 13), 32)
    got = _record(torch, lbm, small)
    want = small.monitors()
    _same(got, want)
    assert got["fluid"] == int(want["fluid"])
    # the entry point rejects a misaligned record address before any work
    rec = torch.zeros(13, dtype=torch.float64, device=small.device)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_monitors_async(small.h, rec.data_ptr() + 4)
    assert e.value.code == -1
    small.close()
