"""Benchmark of the Bingham-fluid LBM stream-collide library on one GPU.

Main line: D3Q27 periodic 256^3 box of random non-overlapping spheres
(radius 8, porosity 0.7, SplitMix64 seed 1), implicitly-regularised operator,
FP64 populations, in-place AA streaming, body force along x, Bingham number
1 (sigma_y = Bi rho g 2R / 4), started from rest, monitors fused every 100
steps.  One step = one fused stream-collide launch over the whole domain.
value = fluid-node updates per second (MLUPS) over the timed steps.

Also reported ("forms"): the PR operator, FP32 and FP16 storage (the FP16
forms on the 384^3 pack, seed 2, without and with the FP64 redo of nodes near
the yield stress), the 4x128x128 D3Q19 duct, and the batched duct sweep, each
with its velocity/flux/plug-volume error against an FP64 run of the same
input at a fixed step (--accuracy-steps from rest, whatever --steps is); and
the creeping-flow cylinder cell of the paper's Table 2 run to steady state,
with its similarity numbers against the printed ones.

Roofline: algorithmic bytes of the step kernel per launch (fluid nodes x
2 Q x 8 B, plus 16 B per fluid node of relaxation time for PR) over its
average duration from HIP events around the timed launches; peak 8 TB/s.
The CPU baseline is the FP64 oracle on the host cores (all of them, and one)
on a few steps of the same workload, with the host's core count and CPU
model.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FORM_GROUPS = ("fp64", "tight", "box", "ab", "lattices", "fp32", "fp16", "duct", "batch", "cylinder")
METRIC = "MLUPS and achieved HBM GB/s (% of peak) vs FP64 form at stated velocity error"
Q = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}
PREC_BYTES = {"FP64": 8, "FP32": 4, "FP16": 2}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_per_node(lattice, op, precision):
    """Bytes one fluid-node update must move: read and write every population
    once, plus read and write the PR relaxation time."""
    b = 2 * Q[lattice] * PREC_BYTES[precision]
    if op == "PR":  # PRI and IR keep no relaxation-time field
        b += 2 * (8 if precision == "FP64" else 4)
    return b


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1610_01388_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hpp", ".hip")):
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def make_domain(lbm, case, precision, scheme="AA", mask=None, pull_form=None, **kw):
    dom = lbm.Domain(case["lattice"], case["dims"], case["periodic"], case["op"], case["nu_p"],
                     case["sigma_y"], m=case["m"], g=case["g"], precision=precision, scheme=scheme, **kw)
    if mask is not None:
        dom.set_mask(mask)  # also resets the state to rest
    if pull_form is not None:
        dom.set_pull_form(pull_form)
    return dom


def timed_run(torch, dom, warmup, steps, mon_every=100):
    dom.set_monitor_interval(mon_every)
    dom.step(warmup)
    torch.cuda.synchronize()
    stream = dom.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    dom.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    return ms, wall


def device_copy_rate(torch, nbytes=2 << 30, reps=10):
    """Read + write bytes per second of a plain device-to-device copy of
    nbytes (torch's copy kernel): what a streaming kernel reaches on this
    GPU, the practical ceiling beside the published peak."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(2):
        b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes * reps / (ms * 1e-3) / 1e9


def phase_times(torch, dom, pairs=20):
    """Mean duration of each AA phase, timed one launch at a time with HIP
    events on the domain's stream (monitors off; the state just advances):
    the pull (neighbour) phase at even times, the local phase at odd ones."""
    dom.set_monitor_interval(0)
    if dom.time % 2:
        dom.step(1)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * pairs)]
    for p in range(pairs):
        ev[3 * p].record(dom.stream)
        dom.step(1)
        ev[3 * p + 1].record(dom.stream)
        dom.step(1)
        ev[3 * p + 2].record(dom.stream)
    torch.cuda.synchronize()
    pull = [ev[3 * p].elapsed_time(ev[3 * p + 1]) for p in range(pairs)]
    loc = [ev[3 * p + 1].elapsed_time(ev[3 * p + 2]) for p in range(pairs)]
    return {"pull_ms": float(np.mean(pull)), "local_ms": float(np.mean(loc))}


def compare(ref, got, axis):
    """Velocity L2-rel, flux rel (along the force axis), plug volume
    (unyielded count) rel."""
    rho_r, u_r, _, uy_r = ref
    rho_g, u_g, _, uy_g = got
    l2 = float(np.linalg.norm(u_g - u_r) / max(np.linalg.norm(u_r), 1e-300))
    fr, fg = u_r[axis].sum(), u_g[axis].sum()
    flux_rel = float(abs(fg - fr) / max(abs(fr), 1e-300))
    pr, pg = int(uy_r.sum()), int(uy_g.sum())
    plug_rel = float(abs(pg - pr) / max(pr, 1))
    return {"velocity_l2_rel": l2, "flux_rel": flux_rel, "plug_volume_rel": plug_rel,
            "unyielded_ref": pr, "unyielded": pg}


def run_form(torch, lbm, name, case, precision, mask, fluid, warmup, steps, ref=None, develop=0, graph=0, **kw):
    """One bench form: from rest, `develop` untimed steps, the moments at that
    time (the accuracy snapshot, compared with `ref` when given), then
    `warmup` untimed and `steps` timed steps.  The snapshot horizon does not
    depend on the timed step count.  graph > 0: steps replayed from captured
    graphs of that many launches."""
    dom = make_domain(lbm, case, precision, mask=mask, **kw)
    if graph:
        dom.set_graph_steps(graph)
    mom = None
    if develop:
        dom.step(develop)
        mom = dom.moments()
    ms, wall = timed_run(torch, dom, warmup, steps)
    mlups = fluid * steps / (ms * 1e-3) / 1e6
    bpn = algorithmic_bytes_per_node(case["lattice"], case["op"], precision)
    gbs = fluid * bpn * steps / (ms * 1e-3) / 1e9
    out = {"form": name, "lattice": case["lattice"], "operator": case["op"], "precision": precision,
           "dims": list(case["dims"]), "fluid_nodes": int(fluid), "steps": steps, "graph_steps": graph,
           "ms_per_step": ms / steps, "MLUPS": mlups, "algorithmic_GBs": gbs,
           "hbm_frac": gbs / HBM_PEAK_GBS, "bytes_per_node": bpn}
    if kw.get("fp64_fallback"):
        out["fallback_band"] = kw.get("fallback_band")
    if kw.get("layout", "COMPACT") == "COMPACT":
        out["neighbour_kernel"] = dom.pull_form()
    if mom is None:
        mom = dom.moments()
    hist = dom.history()
    if hist:
        out["last_monitor"] = {"step": hist[-1]["step"], "flux": float(hist[-1]["flux"][0]),
                               "fallback_nodes": int(hist[-1]["fallback"]),
                               "unyielded": int(hist[-1]["unyielded"])}
    if ref is not None:
        out["error_vs_fp64"] = compare(ref, mom, int(np.argmax(np.abs(case["g"]))))
        out["error_vs_fp64"]["at_step"] = develop
    dom.close()
    torch.cuda.empty_cache()
    return out, mom


def to_steady(dom, every=1000, tol=1e-8, cap=200_000, label=""):
    """Step until the superficial flux changes by at most tol (relative)
    between monitor records every steps apart, or cap steps; returns the
    flux, the steps taken, the last relative change and the residual."""
    dom.set_monitor_interval(every)
    prev, steps, rel = None, 0, None
    while steps < cap:
        dom.step(every)
        steps += every
        h = dom.history()[-1]
        q = float(h["flux"][0])
        if prev is not None:
            rel = abs(q - prev) / max(abs(q), 1e-300)
            if rel <= tol:
                break
        prev = q
        if steps % 20000 == 0:
            log(f"  {label} {steps} steps, flux {q:.9e}, change {rel}")
    return q, steps, rel, float(h["residual"])


def darcy_sweep(torch, lbm, inputs, n, bis, ops, cap):
    """The porous workload run to a steady Darcy flux for a range of Bingham
    numbers, FP32 storage against FP64 (both to their own steady state)."""
    mask, _ = inputs.sphere_pack((n, n, n), 8.0, 0.7, seed=1)
    for op in ops:
        for bi in bis:
            case = inputs.porous_case(op, n=n, Bi=bi)
            row = {"workload": f"D3Q27 {n}^3 sphere pack, porosity 0.7", "operator": op, "Bi": bi,
                   "sigma_y": case["sigma_y"], "m": case["m"], "criterion": "flux change <= 1e-8 per 1000 steps"}
            mom = {}
            for prec in ("FP64", "FP32"):
                dom = make_domain(lbm, case, prec, mask=mask)
                t0 = time.perf_counter()
                q, steps, rel, res = to_steady(dom, cap=cap, label=f"{op} Bi={bi} {prec}")
                torch.cuda.synchronize()
                row[prec] = {"flux": q, "steps": steps, "last_rel_change": rel, "residual": res,
                             "converged": rel is not None and rel <= 1e-8, "seconds": time.perf_counter() - t0}
                mom[prec] = dom.moments()
                dom.close()
                torch.cuda.empty_cache()
            row["fp32_error_vs_fp64"] = compare(mom["FP64"], mom["FP32"], 0)
            print(json.dumps(row), flush=True)


def precision_study(torch, lbm, inputs, n, horizons, bands):
    """Reduced precision against FP64 on the porous workload (seed 2) at
    several times from rest: FP32, FP16 without the FP64 redo, and FP16 with
    the redo of nodes within each relative band around the yield stress.  One
    JSON line per (operator, form): the errors at each horizon, the share of
    nodes the redo took at the last one, and ms per step."""
    mask, _ = inputs.sphere_pack((n, n, n), 8.0, 0.7, seed=2)
    fluid = int((mask == 0).sum())
    forms = [("FP32", {}), ("FP16", {})] + [("FP16", {"fp64_fallback": True, "fallback_band": b}) for b in bands]
    for op in ("IR", "PR"):
        case = inputs.porous_case(op, n=n, Bi=1.0, m=1e4)
        snaps = {}
        dom = make_domain(lbm, case, "FP64", mask=mask)
        done = 0
        for hz in horizons:
            dom.step(hz - done)
            done = hz
            snaps[hz] = dom.moments()
        dom.close()
        torch.cuda.empty_cache()
        log(f"precision study {op}: FP64 reference to step {horizons[-1]}")
        for prec, kw in forms:
            dom = make_domain(lbm, case, prec, mask=mask, fp16_scale_log2=14, **kw)
            dom.set_monitor_interval(100)
            row = {"study": f"D3Q27 {n}^3 sphere pack (seed 2), Bi 1, from rest", "operator": op, "precision": prec,
                   "fp64_redo_band": kw.get("fallback_band"), "fluid_nodes": fluid, "errors": {}}
            done = 0
            for hz in horizons:
                dom.step(hz - done)
                done = hz
                row["errors"][str(hz)] = compare(snaps[hz], dom.moments(), 0)
            hist = dom.history()
            row["redo_share_last"] = hist[-1]["fallback"] / fluid if hist else None
            row["unyielded_share_last"] = hist[-1]["unyielded"] / fluid if hist else None
            ms, _ = timed_run(torch, dom, 0, 200)
            row["ms_per_step"] = ms / 200
            row["MLUPS"] = fluid * 200 / (ms * 1e-3) / 1e6
            dom.close()
            torch.cuda.empty_cache()
            print(json.dumps(row), flush=True)


def run_batch(torch, lbm, cases, precision, warmup, steps, autotune=True, graph_steps=1000):
    """The batched sweep: every case in one batch, stepped by replays of one
    captured graph of graph_steps persistent launches (one per step); tiles
    and work-item order picked by the autotuner."""
    b = lbm.Batch(cases, precision=precision)
    if autotune:
        b.autotune(10)
    b.set_graph_steps(graph_steps)
    b.set_monitor_interval(100)
    b.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    moms = [b.moments(k) for k in range(len(cases))]
    tiles = b.tiles()
    sched = b.schedule()
    mons = b.monitors()
    b.close()
    torch.cuda.empty_cache()
    return ms, moms, tiles, mons, sched


def batch_form(torch, lbm, cases, warmup, steps, graph_steps=1000):
    """FP32 batched sweep with its error against the FP64 batch of the same
    cases (same steps from rest).  Warmup and timed steps are whole graph
    replays when they are multiples of graph_steps."""
    nodes = sum(int(np.prod(c["dims"])) for c in cases)
    bytes_step = sum(int(np.prod(c["dims"])) * algorithmic_bytes_per_node(c["lattice"], c["op"], "FP32")
                     for c in cases)
    ms32, m32, tiles, mons, sched = run_batch(torch, lbm, cases, "FP32", warmup, steps, graph_steps=graph_steps)
    ms64, m64, _, _, _ = run_batch(torch, lbm, cases, "FP64", warmup, steps, graph_steps=graph_steps)
    cat = lambda ms: (np.concatenate([m[0] for m in ms]), np.concatenate([m[1] for m in ms], axis=1), None,
                      np.concatenate([m[3] for m in ms]))
    err = compare(cat(m64), cat(m32), 2)
    # per-simulation flux error over the ducts that still flow in FP64
    rel = []
    for a, c in zip(m64, m32):
        f64, f32 = a[1][2].sum(), c[1][2].sum()
        if abs(f64) > 1e-12 * a[1].shape[1]:
            rel.append(abs(f32 - f64) / abs(f64))
    err["flux_rel_max_per_sim"] = float(max(rel)) if rel else None
    err["flowing_sims"] = len(rel)
    shapes = {}
    for t in tiles:
        shapes[f"{t[0]}x{t[1]}x{t[2]}"] = shapes.get(f"{t[0]}x{t[1]}x{t[2]}", 0) + 1
    ops = {}
    for c in cases:
        key = c["op"] if c["op"] == "IR" else f"PR m={c['m']:g}"
        ops[key] = ops.get(key, 0) + 1
    gbs = bytes_step * steps / (ms32 * 1e-3) / 1e9
    return {"form": f"batched sweep: {len(cases)} D3Q19 ducts FP32", "lattice": "D3Q19", "precision": "FP32",
            "simulations": len(cases), "nodes": nodes, "steps": steps, "ms_per_step": ms32 / steps,
            "MLUPS": nodes * steps / (ms32 * 1e-3) / 1e6, "algorithmic_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "algorithmic_bytes_per_step": bytes_step, "graph_steps": graph_steps, "tiles": shapes,
            "tile_policy": sched[0], "xcd_order": sched[1], "operators": ops,
            "fp64_batch_MLUPS": nodes * steps / (ms64 * 1e-3) / 1e6,
            "nonfinite_sims": int(sum(1 for m in mons if m["nonfinite"])),
            "error_vs_fp64": err}


def cylinder_form(torch, lbm, inputs):
    """Validation form: the creeping-flow cylinder cell of Table 2 (IR,
    sigma_y = 1e-5), from rest to steady state; MLUPS of the whole run and
    the similarity numbers against the printed ones (U = mean over fluid
    nodes)."""
    case = inputs.cylinder_case("IR", sigma_y=1e-5)
    dom = lbm.Domain(case["lattice"], case["dims"], case["periodic"], "IR", case["nu_p"], case["sigma_y"],
                     g=case["g"])
    dom.set_mask(case["mask"])
    fluid = int((case["mask"] == 0).sum())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prev, n = None, 0
    while n < 1_000_000:
        dom.step(2000)
        n += 2000
        U = dom.monitors()["flux"][0]
        if prev is not None and abs(U - prev) <= 1e-9 * abs(U):
            break
        prev = U
    dt = time.perf_counter() - t0
    dom.close()
    U /= 1.0 - case["mask"].mean()
    D, nu, g, sy = case["D"], case["nu_p"], case["g"][0], case["sigma_y"]
    got = {"Re": U * D / nu, "Bn": sy * D / (nu * U), "f": 2 * D * g / U ** 2}
    want = {"Re": 0.802, "Bn": 1.994, "f": 19.890}  # Sec. 4.5.2, Table 2, IR row sigma_y = 1e-5 (read x10)
    return {"form": "cylinder cell 80x80 D2Q9 IR (Table 2 row 2), rest to steady state", "lattice": "D2Q9",
            "precision": "FP64", "fluid_nodes": fluid, "steps": n, "seconds": dt,
            "MLUPS": fluid * n / dt / 1e6, "similarity": got, "paper": want,
            "rel_error": {k: abs(got[k] - want[k]) / want[k] for k in want}}


def host_description():
    """Host cores and CPU model of the machine the CPU baseline runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def oracle_threads():
    """All host cores the process may use (OMP_NUM_THREADS caps it)."""
    host = host_description()
    n = host["usable_cpus"] or 1
    if host["omp_num_threads"]:
        try:
            n = min(n, int(host["omp_num_threads"]))
        except ValueError:
            pass
    return max(1, n)


def time_oracle(case, mask, steps, threads, chunk=None):
    """MLUPS of the FP64 oracle (as it stands) on `steps` steps of a case
    (stepped in chunks with a progress line each, when given)."""
    import oracle
    op = {"PR": oracle.PR, "IR": oracle.IR, "PRI": oracle.PRI}[case["op"]]
    lat = {"D2Q9": 0, "D3Q19": 1, "D3Q27": 2}[case["lattice"]]
    rh = oracle.rheology(op, case["nu_p"], case["sigma_y"], case["m"], 1e-8, 0.25, case["g"])
    used = oracle.set_threads(threads)
    od = oracle.Domain(lat, case["dims"], case["periodic"], rh, mask)
    fluid = int(np.prod(case["dims"])) if mask is None else int((np.asarray(mask) == 0).sum())
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(steps - done, chunk or steps)
        od.step(n)
        done += n
        if chunk:
            log(f"  oracle {case['lattice']} {case['op']}: {done}/{steps} steps on {used} threads, "
                f"{time.perf_counter() - t0:.1f} s")
    dt = time.perf_counter() - t0
    od.close()
    return fluid * steps / dt / 1e6, dt, used


def cpu_baseline(case, mask, fluid):
    """The FP64 oracle (as it stands) on the host cores: one step of the main
    workload on one thread and four steps on every core the process may use
    (about 10-20 s of CPU work in all)."""
    host = host_description()
    one, dt1, _ = time_oracle(case, mask, 1, 1)
    nthr = oracle_threads()
    allc, dtn, used = time_oracle(case, mask, 4, nthr)
    dims = "x".join(str(v) for v in case["dims"])
    return {"value": allc, "unit": "MLUPS", "cores": used, "kind": "oracle",
            "single_core_value": one, "host": host,
            "sample": f"the full {dims} {case['lattice']} {case['op']} FP64 workload ({fluid} fluid nodes): "
                      f"1 step on 1 thread ({dt1:.1f} s) and 4 steps on {used} threads ({dtn:.1f} s), "
                      "plain C with OpenMP over rows, results identical for any thread count"}


def cpu_configs(inputs):
    """The oracle on the two small configurations in full: the D2Q9 4x64
    Bingham channel (20 000 steps, IR and PR) and the D3Q19 4x128x128 duct
    (Bi 0.5, 50 000 steps, IR; all cores in full, one thread over a 1 000-step
    window).  One JSON line each."""
    host = host_description()
    nthr = oracle_threads()
    for op in ("IR", "PR"):
        c = inputs.channel_case(op, H=64, nx=4, Bi=1.0)
        one, dt1, _ = time_oracle(c, None, 20000, 1)
        allc, dtn, used = time_oracle(c, None, 20000, nthr)
        print(json.dumps({"cpu_config": "D2Q9 4x64 Bingham channel, Bi 1, 20000 steps", "operator": op,
                          "MLUPS_1_thread": one, "seconds_1_thread": dt1, "MLUPS_all": allc, "seconds_all": dtn,
                          "threads": used, "host": host}), flush=True)
    duct = inputs.duct_case("IR", side=128, length=4, Bi=0.5)
    allc, dtn, used = time_oracle(duct, None, 50000, nthr, chunk=2500)
    one, dt1, _ = time_oracle(duct, None, 1000, 1, chunk=250)
    print(json.dumps({"cpu_config": "D3Q19 4x128x128 square duct, Bi 0.5, IR", "MLUPS_all_50000_steps": allc,
                      "seconds_all": dtn, "threads": used, "MLUPS_1_thread_1000_steps": one, "seconds_1_thread": dt1,
                      "host": host}), flush=True)


def traffic_from_profile(kernel_hash, per_launch_bytes):
    """HBM traffic of the step kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_d3q27_ir_fp64_aa_porous256.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_hash") != kernel_hash:
        return None
    return d.get("traffic_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-forms", action="store_true", help="main line only")
    ap.add_argument("--only", default=None,
                    help="comma-separated form groups to run (default: all): " + ",".join(FORM_GROUPS))
    ap.add_argument("--accuracy-steps", type=int, default=1000,
                    help="steps from rest at which reduced-precision forms are compared with FP64")
    ap.add_argument("--precision-study", action="store_true",
                    help="instead of the throughput line: FP32 and FP16 (without and with the FP64 redo in several "
                         "bands) against FP64 at several times from rest on the --size pack (seed 2)")
    ap.add_argument("--study-steps", default="1000,5000,20000", help="horizons of --precision-study")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="instead of the throughput line: time the oracle on the two small configurations in full")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched sweep form (for profiling its kernel)")
    ap.add_argument("--layout", default="COMPACT", choices=["COMPACT", "DENSE"],
                    help="population storage layout of the main line")
    ap.add_argument("--darcy", action="store_true",
                    help="instead of the throughput line: the porous workload run to steady Darcy flux for "
                         "Bi in {0.1, 0.316, 1, 3.16, 10}, IR and PR, FP32 against FP64 (one JSON line each)")
    ap.add_argument("--darcy-cap", type=int, default=200_000, help="step cap of each --darcy run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy first (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; decomposing the domain over several GPUs "
              "is not implemented", file=sys.stderr)
        sys.exit(2)

    if args.cpu_configs:
        from paper_1610_01388_amd import inputs
        cpu_configs(inputs)
        return

    import torch
    from paper_1610_01388_amd import inputs, lbm
    torch.cuda.set_device(0)

    if args.precision_study:
        precision_study(torch, lbm, inputs, args.size, [int(v) for v in args.study_steps.split(",")],
                        (0.02, 0.05, 0.2))
        return

    if args.darcy:
        darcy_sweep(torch, lbm, inputs, args.size, (0.1, 0.316, 1.0, 3.16, 10.0), ("IR", "PR"), args.darcy_cap)
        return

    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()

    if args.batch_only:
        log(f"batched sweep only: warmup {args.warmup}, steps {args.steps}")
        g = 1000 if args.steps % 1000 == 0 and args.warmup % 1000 == 0 else 100
        print(json.dumps(batch_form(torch, lbm, inputs.batch_sweep(), args.warmup, args.steps, graph_steps=g)),
              flush=True)
        return

    n = args.size
    log(f"generating {n}^3 sphere pack (R=8, porosity 0.7, seed 1)")
    t0 = time.perf_counter()
    mask, centres = inputs.sphere_pack((n, n, n), 8.0, 0.7, seed=1)
    log(f"  {len(centres)} spheres in {time.perf_counter() - t0:.1f} s, porosity {1 - mask.mean():.4f}")
    fluid = int((mask == 0).sum())
    case = inputs.porous_case("IR", n=n, Bi=1.0)
    case_pr = inputs.porous_case("PR", n=n, Bi=1.0, m=1e4)

    log(f"main: D3Q27 {n}^3 IR FP64 AA {args.layout}, warmup {args.warmup}, steps {args.steps}")
    dom = make_domain(lbm, case, "FP64", mask=mask, layout=args.layout)
    tile = dom.tile()
    nk = dom.pull_form() if args.layout == "COMPACT" else None
    ms, wall = timed_run(torch, dom, args.warmup, args.steps)
    hist = dom.history()
    phases = phase_times(torch, dom) if args.layout == "COMPACT" else None
    dom.close()
    torch.cuda.empty_cache()
    ms_step = ms / args.steps
    mlups = fluid * args.steps / (ms * 1e-3) / 1e6
    bpn = algorithmic_bytes_per_node("D3Q27", "IR", "FP64")
    per_launch = fluid * bpn
    achieved = per_launch / (ms_step * 1e-3) / 1e9
    khash = kernel_source_hash()
    traffic = traffic_from_profile(khash, per_launch) if args.layout == "COMPACT" else None
    copy_gbs = device_copy_rate(torch)
    log(f"  device copy (2 GiB, read + write): {copy_gbs:.0f} GB/s")
    log(f"  {ms_step:.3f} ms/step, {mlups:.1f} MLUPS, {achieved:.0f} GB/s algorithmic")

    result = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"D3Q27 periodic {n}^3 random sphere pack (R=8, porosity 0.7, seed 1), "
                               "IR Bingham operator, Bi=1, FP64, AA in-place streaming, "
                               f"{args.layout.lower()} layout",
                   "lattice": "D3Q27", "operator": "IR", "precision": "FP64", "scheme": "AA",
                   "layout": args.layout,
                   "dims": [n, n, n], "fluid_nodes": fluid, "porosity": float(1 - mask.mean()),
                   "nu_p": case["nu_p"], "sigma_y": case["sigma_y"], "g": list(case["g"]),
                   "tile": list(tile), "neighbour_kernel": nk, "monitor_every": 100,
                   "parity": "velocity L2-rel <= 1e-10 vs the FP64 oracle (tests/test_gpu_parity.py)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": per_launch, "bytes_per_fluid_node": bpn,
                     "kernel": (("k_step_rows" if nk == "ROWS" else "k_pull_slots")
                                + "<D3Q27, IR, FP64, AA pull> and k_local_slots<D3Q27, IR, FP64> "
                                "(AA local)" if args.layout == "COMPACT" else "k_step<D3Q27, IR, FP64, AA pull/local>")
                               + ", mean of the two alternating AA phases",
                     "kernel_source_hash": khash,
                     "device_copy_GBs": copy_gbs, "frac_of_device_copy": achieved / copy_gbs},
    }
    if phases:
        # each AA phase moves the same algorithmic bytes; the pull phase is the slower kernel
        result["roofline"]["phases"] = {
            "pull_ms": phases["pull_ms"], "local_ms": phases["local_ms"],
            "pull_frac": per_launch / (phases["pull_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "local_frac": per_launch / (phases["local_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "method": "HIP events around single launches on the domain's stream, 20 pairs after the timed steps"}
    if hist:
        result["config"]["last_monitor"] = {"step": hist[-1]["step"], "flux": float(hist[-1]["flux"][0]),
                                            "mass": hist[-1]["mass"], "umax": hist[-1]["umax"],
                                            "unyielded": int(hist[-1]["unyielded"])}

    forms = []
    groups = set(FORM_GROUPS if args.only is None else args.only.split(","))
    unknown = groups - set(FORM_GROUPS)
    if unknown:
        sys.exit(f"bench.py: unknown form groups {sorted(unknown)}; known: {','.join(FORM_GROUPS)}")
    if args.no_forms:
        groups = set()
    W, K, H = args.warmup, min(args.steps, 500), args.accuracy_steps
    ref_ir = ref_pr = None
    if groups & {"fp64", "fp32", "ab"}:
        log(f"forms: FP64 references (compact layout), accuracy snapshot at step {H}")
        f64_ir, ref_ir = run_form(torch, lbm, "IR FP64", case, "FP64", mask, fluid, W, K, develop=H)
        f64_pr, ref_pr = run_form(torch, lbm, "PR FP64", case_pr, "FP64", mask, fluid, W, K, develop=H)
        forms += [f64_ir, f64_pr]
    if "fp64" in groups:
        log("forms: dense layout, PRI, IRHB")
        forms.append(run_form(torch, lbm, "IR FP64 dense layout", case, "FP64", mask, fluid, W, K, ref=ref_ir,
                              develop=H, layout="DENSE")[0])
        case_pri = dict(case_pr, op="PRI")
        forms.append(run_form(torch, lbm, "PRI FP64 (implicit tau update, no tau field)", case_pri, "FP64", mask,
                              fluid, W, K)[0])
        case_hb = dict(case, op="IRHB")
        forms.append(run_form(torch, lbm, "IRHB FP64 (Herschel-Bulkley, n = 0.5, K = nu_p)", case_hb, "FP64", mask,
                              fluid, W, K, hb_n=0.5)[0])
    if "tight" in groups:
        log("forms: tight medium (overlapping spheres, porosity 0.15): row-segment vs slot neighbour kernel")
        mask_t, _ = inputs.overlapping_spheres((n, n, n), 8.0, 0.15, seed=1)
        fl_t = int((mask_t == 0).sum())
        tight_rows, ref_t = run_form(torch, lbm, "IR FP64 tight medium, row-segment kernel", case, "FP64", mask_t,
                                     fl_t, W, K, pull_form="ROWS")
        tight_auto, _ = run_form(torch, lbm, "IR FP64 tight medium, default kernel choice", case, "FP64", mask_t,
                                 fl_t, W, K, ref=ref_t)
        forms += [tight_rows, tight_auto]
        del ref_t, mask_t
    if "box" in groups:
        log("forms: all-fluid periodic box of the same size (ceiling of this access pattern)")
        forms.append(run_form(torch, lbm, "IR FP64 all-fluid periodic box (ceiling)", case, "FP64",
                              np.zeros(n ** 3, dtype=np.uint8), n ** 3, W, K)[0])
    if "ab" in groups:
        log("forms: A/B streaming")
        forms.append(run_form(torch, lbm, "IR FP64 A/B streaming (two copies)", case, "FP64", mask, fluid, W, K,
                              ref=ref_ir, develop=H, scheme="AB")[0])
    if "lattices" in groups:
        log("forms: the D3Q19 and D2Q9 lattices at HBM scale")
        case19 = dict(case, lattice="D3Q19")
        forms.append(run_form(torch, lbm, "IR FP64 D3Q19, same pack", case19, "FP64", mask, fluid, W, K)[0])
        cell = inputs.cylinder_case("IR", sigma_y=1e-5)
        tiles = 51
        mask2 = np.tile(cell["mask"].reshape(80, 80), (tiles, tiles)).reshape(-1)
        case2 = dict(cell, dims=(80 * tiles, 80 * tiles, 1))
        forms.append(run_form(torch, lbm, f"IR FP64 D2Q9, cylinder array {tiles}x{tiles} cells "
                              f"({80 * tiles}^2, Table 2 cell)", case2, "FP64", mask2, int((mask2 == 0).sum()),
                              W, K)[0])
        del mask2
    if "fp32" in groups:
        log(f"forms: FP32 storage and collision, errors at step {H}")
        forms.append(run_form(torch, lbm, "IR FP32", case, "FP32", mask, fluid, W, K, ref=ref_ir, develop=H)[0])
        forms.append(run_form(torch, lbm, "PR FP32", case_pr, "FP32", mask, fluid, W, K, ref=ref_pr, develop=H)[0])
    del ref_ir, ref_pr
    if "fp16" in groups:
        n4 = 384 if n == 256 else n
        log(f"forms: FP16 storage without and with the FP64 redo near the yield stress, {n4}^3 pack (seed 2), "
            f"errors at step {H}")
        mask4, _ = inputs.sphere_pack((n4, n4, n4), 8.0, 0.7, seed=2)
        fl4 = int((mask4 == 0).sum())
        for op in ("IR", "PR"):
            c4 = inputs.porous_case(op, n=n4, Bi=1.0, m=1e4)
            r64, ref4 = run_form(torch, lbm, f"{op} FP64 {n4}^3", c4, "FP64", mask4, fl4, W, K, develop=H)
            forms.append(r64)
            forms.append(run_form(torch, lbm, f"{op} FP16 {n4}^3", c4, "FP16", mask4, fl4, W, K, ref=ref4,
                                  develop=H, fp16_scale_log2=14)[0])
            forms.append(run_form(torch, lbm, f"{op} FP16 + FP64 redo within 5% of the yield stress {n4}^3", c4,
                                  "FP16", mask4, fl4, W, K, ref=ref4, develop=H, fp64_fallback=True,
                                  fallback_band=0.05, fp16_scale_log2=14)[0])
            del ref4
        del mask4
    if "duct" in groups:
        # small and cache-resident: MLUPS only; launch-bound, so each precision
        # is timed with eager launches and with replays of 100-step graphs
        # (1000 steps to develop, 100 warmup, 500 timed: whole replays,
        # whatever --steps is)
        log("forms: D3Q19 4x128x128 duct, eager launches and 100-step graph replays")
        duct = inputs.duct_case("IR", side=128, length=4, Bi=0.5)
        dfl = 128 * 128 * 4
        d64, dref = run_form(torch, lbm, "duct D3Q19 IR FP64", duct, "FP64", None, dfl, 100, 500, develop=1000)
        g64, _ = run_form(torch, lbm, "duct D3Q19 IR FP64, 100-step graphs", duct, "FP64", None, dfl, 100, 500,
                          ref=dref, develop=1000, graph=100)
        d32, _ = run_form(torch, lbm, "duct D3Q19 IR FP32", duct, "FP32", None, dfl, 100, 500, ref=dref,
                          develop=1000)
        g32, _ = run_form(torch, lbm, "duct D3Q19 IR FP32, 100-step graphs", duct, "FP32", None, dfl, 100, 500,
                          ref=dref, develop=1000, graph=100)
        forms += [d64, g64, d32, g32]
    if "batch" in groups:
        log("forms: batched sweep, 256 D3Q19 ducts (sides 32..160, length 4), FP32 vs FP64, 1000-step graph")
        forms.append(batch_form(torch, lbm, inputs.batch_sweep(), 1000, 1000))
    if "cylinder" in groups:
        log("forms: cylinder-array validation cell (Table 2), rest to steady state")
        forms.append(cylinder_form(torch, lbm, inputs))
    result["forms"] = forms

    if not args.no_cpu:
        log("cpu baseline: oracle on one thread and on all host cores, main workload")
        result["cpu_baseline"] = cpu_baseline(case, mask, fluid)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
