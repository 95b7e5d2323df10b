"""Seeded input generators (no lattice Boltzmann arithmetic in them)."""
import json
import os

import numpy as np

from paper_1610_01388_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_splitmix64_reference_vector():
    ref = GOLD["splitmix64_seed_1234567"]["value"]
    r = inputs.SplitMix64(1234567)
    assert [r.next_u64() for _ in range(5)] == ref
    assert [int(v) for v in inputs.splitmix64_array(1234567, 5)] == ref
    assert [int(v) for v in inputs.splitmix64_array(1234567, 3, offset=2)] == ref[2:]


def test_uniform_array_range():
    u = inputs.uniform_array(7, 10000, -1.0, 1.0)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.05


def test_sphere_pack_properties():
    n, R = 64, 8.0
    mask, centres = inputs.sphere_pack((n, n, n), R, 0.7, seed=1)
    assert mask.dtype == np.uint8 and mask.size == n ** 3
    por = 1.0 - mask.mean()
    assert por <= 0.7
    # the last sphere crossed the target: without it porosity was above 0.7
    assert por > 0.7 - 2200.0 / n ** 3
    # centres pairwise at least 2R apart (minimum image)
    d = centres[:, None, :] - centres[None, :, :]
    d -= n * np.round(d / n)
    dist = np.sqrt((d ** 2).sum(-1)) + np.eye(len(centres)) * 1e9
    assert dist.min() >= 2 * R
    # voxel rule: a voxel is solid iff some centre is within R (minimum image)
    m3 = mask.reshape(n, n, n)
    rng = np.random.default_rng(0)
    for _ in range(300):
        z, y, x = rng.integers(0, n, 3)
        dd = centres - np.array([x, y, z])
        dd -= n * np.round(dd / n)
        assert m3[z, y, x] == int(((dd ** 2).sum(1) <= R * R).any())
    # deterministic
    mask2, _ = inputs.sphere_pack((n, n, n), R, 0.7, seed=1)
    assert np.array_equal(mask, mask2)


def test_overlapping_spheres_properties():
    n, R = 48, 5.0
    mask, centres = inputs.overlapping_spheres((n, n, n), R, 0.15, seed=3)
    por = 1.0 - mask.mean()
    assert por <= 0.15
    # without the last sphere the porosity was still above the target
    m3 = np.zeros((n, n, n), dtype=bool)
    for c in centres[:-1]:
        inputs._stamp_sphere(m3, c, R)
    assert 1.0 - m3.mean() > 0.15
    # Boolean model: porosity exp(-k v / N) for k spheres of voxel volume v
    v = 4.0 / 3.0 * np.pi * R ** 3
    assert abs(np.log(por) + len(centres) * v / n ** 3) < 0.05 * len(centres) * v / n ** 3
    # voxel rule as for the non-overlapping pack (minimum image)
    mm = mask.reshape(n, n, n)
    rng = np.random.default_rng(1)
    for _ in range(300):
        z, y, x = rng.integers(0, n, 3)
        dd = centres - np.array([x, y, z])
        dd -= n * np.round(dd / n)
        assert mm[z, y, x] == int(((dd ** 2).sum(1) <= R * R).any())
    assert np.array_equal(mask, inputs.overlapping_spheres((n, n, n), R, 0.15, seed=3)[0])


def test_batch_sweep_recipe():
    cases = inputs.batch_sweep()
    assert len(cases) == 256
    sides = [c["dims"][0] for c in cases]
    assert min(sides) >= 32 and max(sides) <= 160
    ops = {(c["op"], c["m"]) for c in cases}
    assert ops == {("PR", 1e3), ("PR", 1e4), ("PR", 1e5), ("IR", 0.0)}
