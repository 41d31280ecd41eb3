#!/usr/bin/env python3
"""Benchmark: D_ij nonzeros/s and ms per 9-field plan on one MI355X.

One step = the whole plain path for one plan of the 128^3 slab workload
(9 coplanar beams 40 deg apart, 30 x 30 beamlets of 0.5 cm, 8100 rows):
  fspb_plan_create  (FP64 beamlet geometry, VOI row bounds, pinned record image)
  fspb_raytrace     (record upload, density mask + radiological-depth tables)
  fspb_dose_coeffs  (count, scan, fill queued behind them, 8-byte nnz read)
  fspb_plan_destroy
The density grid, the output buffers and the workspaces are resident in HBM
before the timed region.  Consecutive steps alternate between two streams,
each with its own workspace and CSR arrays (--pipeline 2), so that one
plan's upload, trace and count overlap the previous plan's fill, as a caller
computing plan after plan would run them: `value` = nonzeros produced per
second of wall clock over the K timed steps (whole-job throughput) and
`ms_per_step` = wall clock per plan in that loop.  `ms_per_step_one_stream`
is the same loop on one stream (one plan at a time), and
`device_ms_per_plan` the sum of the kernels' HIP-event times of one plan
(the paper's T_GPU).

Printed as one JSON line.  Besides the contract fields it carries
`roofline` (the fill kernel: 8 bytes written per nonzero over its
HIP-event duration, against 8 TB/s), `cpu_baseline` (the FP64 oracle on a
bounded sample of the same workload, on this host's cores),
`error_vs_oracle` (the timed plan's CSR against the oracle's rows of that
sample, and its depth tables against the oracle's), per-kernel times, and
beside the default workload the pelvis (`pelvis`, with its own error against
the oracle over every row), the 32-plan batch (`batch32`), Eq. 1 (`eq1`),
the rows beyond the plain path (`next_rows`) and the learned surrogate checked
against the oracle (`surrogate`).
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "D_ij nonzeros/s + ms per 9-field plan; surrogate vs analytic at <=0.5% error"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", type=int, default=1, choices=[1, 2, 3],
                    help="1: 128^3 slab (default); 2: 256x256x100 pelvis; "
                         "3: 32 uneven plans as one captured graph")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target duration of the oracle sample (0 disables)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pipeline", type=int, default=2, choices=[1, 2, 3],
                    help="plans in flight: step k runs on stream k mod P with its own workspace and "
                         "outputs, so one plan's trace and count overlap another's fill")
    ap.add_argument("--no-eq1", action="store_true", help="skip the Eq. 1 (dose, gradient, transpose) timings")
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the pelvis and 32-plan batch measurements beside the default workload "
                         "(profiling runs of the headline plan)")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the trilinear-table, tabulated-kernel and chunked-computation timings")
    ap.add_argument("--table1", action="store_true",
                    help="the paper's water-phantom study (Table 1, cases 1-7): one JSON line, context only")
    ap.add_argument("--surrogate-epochs", type=int, default=None,
                    help="training epochs of the kernel surrogate compared with the analytic "
                         "fill on the pelvis workload (0 skips it; default: 800 beside the default workload)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes three times (reference "
                         "dispatch for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def copy_calibration(nbytes):
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "dispatches": 3}), flush=True)


def fill_profile(workload):
    """Committed rocprofv3 counter figures of the fill (profiles/fill_traffic.json), if they
    were taken on this workload with the current fill sources; else None."""
    path = os.path.join(ROOT, "profiles", "fill_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_0908_4417_amd import build as b
    if d.get("kernel_source_sha") != b.kernel_source_sha() or d.get("workload") != workload:
        return None
    return d


def traffic_from_profile(kernel_name, workload):
    """HBM bytes per fill launch from committed rocprofv3 counter summaries, if current."""
    d = fill_profile(workload)
    return None if d is None else d.get("bytes_per_launch")


# VALU issue peak: 256 CUs x 4 SIMDs x one wave64 instruction per 4 cycles x 2.4 GHz, in lane
# instructions per second (packed FP32 is kept out of the code objects)
VALU_PEAK_LANE_INSTR = 256 * 4 * 16 * 2.4e9


def valu_roofline(workload, fill_s):
    """The fill against its real bound: VALU instructions per launch (SQ_INSTS_VALU from the
    committed counter profile) over the fill time measured here."""
    d = fill_profile(workload)
    if d is None or not d.get("valu_insts_per_launch"):
        return None
    achieved = d["valu_insts_per_launch"] * 64 / fill_s
    return {"bound": "alu", "achieved": round(achieved / 1e12, 2), "peak": round(VALU_PEAK_LANE_INSTR / 1e12, 2),
            "unit": "T VALU lane-instructions/s", "frac": round(achieved / VALU_PEAK_LANE_INSTR, 4),
            "valu_insts_per_nonzero": round(d["valu_insts_per_launch"] * 64 / d["algorithmic_bytes_per_launch"] * 8, 1)}


def _gpu_rows(indptr_h, indices, values, sel):
    """Host copies of the GPU CSR rows `sel` (ascending), gathered on the device."""
    import torch
    a, b = indptr_h[sel], indptr_h[sel + 1]
    pos = np.concatenate([np.arange(x, y, dtype=np.int64) for x, y in zip(a, b)] + [np.zeros(0, np.int64)])
    p = torch.from_numpy(pos).to(indices.device)
    return indices[p].cpu().numpy(), values[p].cpu().numpy().astype(np.float64), np.diff(np.concatenate([[0], np.cumsum(b - a)]))


class OracleError:
    """Error of the GPU rows against the oracle's, accumulated chunk by chunk: the 1e-4
    relative bar is applied to entries above 1 % of the largest entry (taken as 0.99 % of
    the GPU's largest, which is the larger set once the two maxima agree to 1e-4), eps is
    the mean absolute difference over common entries (the paper's measure, Sec. 3.1)."""

    def __init__(self, gmax):
        self.thr = 0.0099 * gmax
        self.gmax, self.omax = gmax, 0.0
        self.max_rel, self.abs_sum, self.n, self.rows, self.mismatch = 0.0, 0.0, 0, 0, 0

    def add(self, off, oidx, oval, gidx, gval, gcnt):
        self.rows += len(off) - 1
        if len(oval):
            self.omax = max(self.omax, float(oval.max()))
        if np.array_equal(gcnt, np.diff(off)) and np.array_equal(gidx, oidx):
            o, g = oval, gval
        else:
            gs = np.concatenate([[0], np.cumsum(gcnt)])
            os_, gs_ = [], []
            for r in range(len(off) - 1):
                a, b = oidx[off[r]:off[r + 1]], gidx[gs[r]:gs[r + 1]]
                common, ia, ib = np.intersect1d(a, b, assume_unique=True, return_indices=True)
                self.mismatch += len(a) + len(b) - 2 * len(common)
                os_.append(oval[off[r]:off[r + 1]][ia])
                gs_.append(gval[gs[r]:gs[r + 1]][ib])
            o, g = np.concatenate(os_), np.concatenate(gs_)
        d = np.abs(g - o)
        self.abs_sum += float(d.sum())
        self.n += len(o)
        big = o > self.thr
        if big.any():
            self.max_rel = max(self.max_rel, float((d[big] / o[big]).max()))

    def result(self):
        return {"max_rel": float(f"{self.max_rel:.3e}"), "eps": float(f"{self.abs_sum / max(self.n, 1):.3e}"),
                "rows": self.rows, "entries": self.n, "pattern_mismatches": self.mismatch,
                "max_entry_rel_diff": float(f"{abs(self.gmax - self.omax) / max(self.omax, 1e-300):.3e}"),
                "bar": "max_rel <= 1e-4 on entries above 1 % of the maximum (0.99 % of the GPU maximum); "
                       "pattern mismatches only within 1e-4 cm of the cutoff (checked in the tests)"}


def cpu_baseline(prob, target_s, n_beamlets, gpu_csr=None):
    """Oracle on a seeded sample of beamlet rows, scaled to nonzeros per second.

    Rows are taken in a seeded random order, 64 at a time (count, then rows,
    both timed), until about ``target_s`` seconds have passed; memory stays
    bounded by one chunk.  With ``gpu_csr`` (indptr, indices, values on the
    device) the same rows of the GPU's CSR are compared with the oracle's,
    outside the timed calls.
    """
    import oracle
    ora = oracle.OraclePlan(prob)
    order = np.random.default_rng(12345).permutation(n_beamlets)
    err = None
    if gpu_csr is not None:
        indptr_h = gpu_csr[0].cpu().numpy()
        err = OracleError(float(gpu_csr[2].max().item()))
    nz = 0
    done = 0
    dt = 0.0
    while done < n_beamlets and dt < target_s:
        sel = np.sort(order[done:done + 64])
        t0 = time.perf_counter()
        off, idx, val = ora.rows(sel, ora.counts_of(sel))
        dt += time.perf_counter() - t0
        nz += int(off[-1])
        done += len(sel)
        if err is not None:
            gi, gv, gc = _gpu_rows(indptr_h, gpu_csr[1], gpu_csr[2], sel.astype(np.int64))
            err.add(off, idx, val, gi, gv, gc)
    table_err = None
    if err is not None:
        # the plan's depth tables (Sec. 2.2) against the oracle's, in cm
        from paper_0908_4417_amd import Plan
        plan = Plan(prob, "cuda:0")
        plan.raytrace()
        tab, toff = plan.tables()
        otab, ooff = ora.tables()
        if np.array_equal(toff, ooff):
            table_err = float(f"{np.max(np.abs(tab.astype(np.float64) - otab)):.3e}")
        del plan
    cores = oracle.max_threads()
    # the same oracle on one thread, over the first 64 rows of the same order
    sel = np.sort(order[:64])
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        off, idx, val = ora.rows(sel, ora.counts_of(sel))
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(cores)
    out = {"value": round(nz / dt, 1), "unit": "D_ij nonzeros/s", "cores": cores,
           "kind": "oracle",
           "sample": f"{done} of {n_beamlets} beamlet rows (seeded order), {nz} nonzeros in {dt:.1f} s; "
                     f"FP64 C oracle, OpenMP over rows",
           "one_thread": {"value": round(int(off[-1]) / dt1, 1), "unit": "D_ij nonzeros/s",
                          "sample": f"first 64 rows of the same order, {int(off[-1])} nonzeros in {dt1:.2f} s"}}
    res = None
    if err is not None:
        res = err.result()
        res["max_table_err_cm"] = table_err      # None if the table layouts differ
    return out, res


def oracle_error(prob, gpu_csr):
    """Every row of a plan's GPU CSR against the oracle's (64 rows at a time), as the
    cpu_baseline leg does for the timed plan."""
    import oracle
    ora = oracle.OraclePlan(prob)
    indptr_h = gpu_csr[0].cpu().numpy()
    err = OracleError(float(gpu_csr[2].max().item()))
    n = len(indptr_h) - 1
    for j0 in range(0, n, 64):
        sel = np.arange(j0, min(j0 + 64, n))
        off, idx, val = ora.rows(sel, ora.counts_of(sel))
        gi, gv, gc = _gpu_rows(indptr_h, gpu_csr[1], gpu_csr[2], sel.astype(np.int64))
        err.add(off, idx, val, gi, gv, gc)
    return err.result()


def surrogate_comparison(epochs, cpu=True):
    """Train the kernel surrogate on the GPU and compare its fused fill with the analytic fill.

    Workload: the 256 x 256 x 100 pelvis (9 beams, 0.25 cm beamlets).  The
    surrogate is trained on 1e7 seeded samples of the analytic kernel (drawn
    uniformly in the square-root feature coordinates, beamlet side
    log-uniform, 10 % at zero depth); both fills are timed with HIP events.
    With ``cpu`` the oracle computes every row of the plan (FP64), and both
    fills are compared with it: the dose of a uniform fluence (Eq. 1; the
    surrogate's target is a maximum dose error of 0.5 % of the maximum dose)
    and every coefficient (maximum and RMS error over entries above 1 % of the
    maximum, relative to the largest coefficient).
    """
    import torch
    import fspb_inputs as fi
    import paper_0908_4417_amd as m
    from paper_0908_4417_amd import Plan, Surrogate
    prob = fi.make_config(4)
    dev = "cuda:0"
    n_samples = fi.SURROGATE_SAMPLES
    sur = Surrogate(prob.kernel, fi.surrogate_init(5), max_batch=16384)
    raw = fi.surrogate_samples(n_samples, seed=5, **fi.SURROGATE_RECIPE).astype(np.float32)
    f, t = sur.targets(torch.from_numpy(raw).to(dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = sur.train(f, t, epochs=epochs, seed=5, **fi.SURROGATE_TRAINING)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del f, t
    plan = Plan(prob, dev)
    m.fspb_plan_set_timing(plan.handle, 1)

    def run():
        times = []
        for _ in range(4):
            csr = plan.compute()
            times.append(m.fspb_plan_get_timing(plan.handle).fill_ms)
        dose = csr.dose(torch.ones(plan.n_beamlets, dtype=torch.float32, device=dev)).double()
        torch.cuda.synchronize()
        return min(times[1:]), dose, csr.values.clone()

    ta, Da, va = run()
    plan.set_surrogate(sur)
    ts, Ds, vs = run()
    out = {"workload": "surrogate_on_pelvis256x256x100_9beam_5184bl", "samples": n_samples, "epochs": epochs,
           "train_s": round(train_s, 3), "final_loss": float(losses[-1]),
           "fill_ms_analytic": round(ta, 4), "fill_ms_surrogate": round(ts, 4),
           "surrogate_time_over_analytic": round(ts / ta, 2),
           "surrogate_faster": bool(ts < ta)}
    if cpu:
        import oracle
        ora = oracle.OraclePlan(prob)
        indptr_h = plan.indptr.cpu().numpy()
        dose_o = np.zeros(plan.n_voxels)
        worst = {"a": 0.0, "s": 0.0}
        sq = {"a": [], "s": []}
        for j0 in range(0, ora.n_beamlets, 64):
            sel = np.arange(j0, min(j0 + 64, ora.n_beamlets))
            off, oidx, oval = ora.rows(sel)
            np.add.at(dose_o, oidx, oval)
            a, b = int(indptr_h[sel[0]]), int(indptr_h[sel[-1] + 1])
            # the surrogate fill keeps the analytic pattern (asserted in the tests)
            for key, vals in (("a", va), ("s", vs)):
                d = np.abs(vals[a:b].cpu().numpy().astype(np.float64) - oval)
                worst[key] = max(worst[key], float(d.max()) if len(d) else 0.0)
                sq[key].append((oval, d))
        omax = max(float(o.max()) for o, _ in sq["a"] if len(o))
        dmax = dose_o.max()
        inside = dose_o > 0
        for key, D, label in (("a", Da, "analytic"), ("s", Ds, "surrogate")):
            dd = np.abs(D.cpu().numpy() - dose_o)
            big = np.concatenate([d[o > 0.01 * omax] for o, d in sq[key]])
            out[label + "_vs_oracle"] = {
                "max_dose_err": float(f"{dd.max() / dmax:.4e}"),
                "rms_dose_err": float(f"{np.sqrt(np.mean(dd[inside] ** 2)) / dmax:.4e}"),
                "max_coeff_err": float(f"{worst[key] / omax:.4e}"),
                "rms_coeff_err": float(f"{np.sqrt(np.mean(big ** 2)) / omax:.4e}")}
        out["dose_target"] = "max dose error <= 0.5 % of the maximum dose (uniform fluence, Eq. 1)"
        out["dose_target_met"] = bool(out["surrogate_vs_oracle"]["max_dose_err"] <= 5e-3)
    return out


def eq1_timings(indptr, indices, values, n_voxels, n_beamlets, reps=5):
    """Device times (HIP events, launch stream) of Eq. 1 on the plan's D_ij.

    fluence_dose: dose = D w on the beamlet-row CSR (atomics); gradient:
    g = D^T r; transpose: the voxel-row CSR (device time of the whole call,
    which runs without host synchronisation); voxel_dose: D w on the voxel rows
    (no atomics).  Bytes per call: 8 per nonzero plus the vectors.
    """
    import torch
    from paper_0908_4417_amd import CSR
    dev = indices.device
    csr = CSR(indptr, indices, values, n_voxels)
    w = torch.rand(n_beamlets, device=dev)
    r = torch.rand(n_voxels, device=dev)
    stream = torch.cuda.current_stream(dev)

    def timed(fn, reps=reps):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"fluence_dose_ms": timed(lambda: csr.dose(w)), "gradient_ms": timed(lambda: csr.gradient(r))}
    t = csr.transpose()
    out["transpose_ms"] = timed(lambda: csr.transpose(), reps=3)   # device time (no host synchronisation)
    out["voxel_dose_ms"] = timed(lambda: t.dose(w))
    d1, d2 = csr.dose(w).double(), t.dose(w).double()
    out["voxel_vs_atomic_max_rel"] = (d1 - d2).abs().max().item() / d1.abs().max().item()
    nnz = int(indices.numel())
    for k in ("fluence_dose", "gradient", "voxel_dose"):
        out[k + "_GBps"] = round(8.0 * nnz / (out[k + "_ms"] * 1e-3) / 1e9, 1)
    del t
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in out.items()}


def next_rows_timings(prob, reps=5):
    """Device times of the rows beyond the plain path on the same workload.

    trilinear: the paper's trilinear-sampled depth table (raytrace and fill);
    tables: the general form of Eq. 2-3 (three terms, depth-tabulated c and A(theta, d));
    chunks: D computed beam by beam under a one-beam memory budget (wall clock,
    including the one count pass), against one-shot computation.
    """
    import dataclasses
    import torch
    import fspb_inputs as fi
    import paper_0908_4417_amd as m
    from paper_0908_4417_amd import Plan

    def timed_plan(problem):
        plan = Plan(problem, "cuda:0")
        m.fspb_plan_set_timing(plan.handle, 1)
        ts = []
        for _ in range(reps + 1):
            csr = plan.compute()
            ts.append(m.fspb_plan_get_timing(plan.handle))
        torch.cuda.synchronize()
        med = lambda k: float(np.median([getattr(t, k) for t in ts[1:]]))
        out = {"nnz": csr.nnz, "raytrace_ms": round(med("raytrace_ms"), 4), "fill_ms": round(med("fill_ms"), 4),
               "device_ms": round(sum(med(k) for k in ("prep_ms", "raytrace_ms", "count_ms", "scan_ms", "fill_ms")), 4)}
        del csr, plan
        torch.cuda.empty_cache()
        return out

    k = prob.kernel
    res = {"trilinear": timed_plan(dataclasses.replace(prob, kernel=dataclasses.replace(k, depth="trilinear")))}
    kt = dataclasses.replace(k, weight=[0.0] * 3, sigma0=[1.0] * 3, sigma_slope=[0.0] * 3, width_scale=[1.0] * 3,
                             tables=fi.synthetic_tables(71, k))
    res["tables_3_terms"] = timed_plan(dataclasses.replace(prob, kernel=kt))
    plan = Plan(prob, "cuda:0")
    plan.compute()
    torch.cuda.synchronize()
    walls = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.compute()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    one_shot = min(walls)
    nnz = plan.nnz
    budget = int(8 * nnz / len(prob.beams) * 1.05)
    walls = []
    pieces = 0
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pieces = 0
        for _j0, _j1, _c in plan.chunks(budget):
            pieces += 1
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    res["chunks"] = {"budget_bytes": budget, "pieces": pieces, "wall_ms": round(1e3 * min(walls), 4),
                     "one_shot_wall_ms": round(1e3 * one_shot, 4)}
    del plan
    torch.cuda.empty_cache()
    return res


# Table 1 of the paper (Tesla C1060, single precision): N'_voxel and T_GPU in seconds, context only
PAPER_TABLE1 = {1: (0.864e7, 0.06), 2: (1.80e7, 0.10), 3: (3.23e7, 0.18), 4: (5.27e7, 0.30),
                5: (4.97e7, 0.29), 6: (4.70e7, 0.27), 7: (4.39e7, 0.24)}


def bench_table1(args):
    """The seven water-phantom cases of Table 1 (30 cm cube, 5 beams, 10 x 10 cm field):
    coefficients and device time per plan on this GPU beside the paper's figures."""
    import torch
    import fspb_inputs as fi
    import paper_0908_4417_amd as m
    from paper_0908_4417_amd import Plan
    rows = []
    for case in range(1, 8):
        plan = Plan(fi.table1_case(case), "cuda:0")
        m.fspb_plan_set_timing(plan.handle, 1)
        times, walls = [], []
        for _ in range(max(args.steps, 3)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            csr = plan.compute()
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            t = m.fspb_plan_get_timing(plan.handle)
            times.append(t.prep_ms + t.raytrace_ms + t.count_ms + t.scan_ms + t.fill_ms)
        n_ref, t_ref = PAPER_TABLE1[case]
        rows.append({"case": case, "nnz": csr.nnz, "paper_nnz": n_ref, "device_ms": round(min(times[1:]), 4),
                     "wall_ms": round(1e3 * min(walls[1:]), 4), "paper_gpu_ms": 1e3 * t_ref,
                     "nnz_per_s": round(csr.nnz / (min(times[1:]) * 1e-3), 1)})
        del csr, plan
    print(json.dumps({"metric": "Table 1 water phantom: coefficients and device time per plan",
                      "data": "synthetic", "context": "paper: Tesla C1060, single precision", "cases": rows}),
          flush=True)


def batch_workload(steps, warmup):
    """32 plans of uneven size, computed by one graph launch per step (tuned first).

    Device time of the graph launches by HIP events on the launch stream,
    nonzeros of all plans, the tuned fill shape and the fill's share of HBM
    (8 B per nonzero over the tuned fill time).
    """
    import torch
    import fspb_inputs as fi
    from paper_0908_4417_amd import Plan, Batch
    probs = fi.batched_configs(n_plans=32)
    plans = [Plan(p, "cuda:0") for p in probs]
    batch = Batch(plans)
    cfg = batch.tune()
    total = int(sum(batch.nnz))
    for _ in range(warmup):
        batch.run()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        batch.run()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert batch.check() == 0
    dev_ms = e0.elapsed_time(e1) / steps
    achieved = 8.0 * total / (cfg.fill_ms * 1e-3) / 1e9
    out = {"workload": fi.CONFIG_NAMES[3], "plans": len(plans), "beamlets": int(sum(p.n_beamlets for p in plans)),
           "nnz": total, "graph_ms": round(dev_ms, 4), "ms_per_step_wall": round(1e3 * wall / steps, 4),
           "nnz_per_s": round(total / (dev_ms * 1e-3), 1),
           "tuned_fill": {"waves_per_group": cfg.waves_per_group, "groups_per_cu": cfg.groups_per_cu,
                          "order": "longest-first" if cfg.order == 0 else "plan", "tile_rows": cfg.tile_rows,
                          "beamlets_per_item": cfg.beamlets_per_item, "fill_ms": round(cfg.fill_ms, 4)},
           "fill_roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": "kp_fill",
                             "bytes_per_launch": 8.0 * total}}
    del batch, plans
    torch.cuda.empty_cache()
    return out, total, wall


def bench_batch(args):
    """The 32-plan batch as the timed workload (--workload 3)."""
    import fspb_inputs as fi
    res, total, wall = batch_workload(args.steps, args.warmup)
    out = {
        "metric": METRIC, "value": round(total * args.steps / wall, 1), "unit": "D_ij nonzeros/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": fi.CONFIG_NAMES[3], "plans": res["plans"], "beamlets": res["beamlets"],
                   "nnz": total},
        "roofline": res["fill_roofline"],
        "graph_device_ms": res["graph_ms"],
        "tuned_fill": res["tuned_fill"],
    }
    print(json.dumps(out), flush=True)


def plan_workload(k, steps, warmup, P):
    """One single-plan workload timed as the bench's steps (see the module docstring).

    Returns (summary dict, the plan's CSR (indptr, indices, values) on the device,
    the problem).  Device times per kernel come from HIP events on the launch
    stream in a separate one-stream pass (medians over the steps).
    """
    import torch
    import fspb_inputs as fi
    import paper_0908_4417_amd as m
    from paper_0908_4417_amd.plan import _structs

    dev = torch.device("cuda:0")
    prob = fi.make_config(k)
    density = torch.from_numpy(prob.grid.density).to(dev)
    grid, beams, kern, _pdd = _structs(prob, density.data_ptr())
    nb = len(prob.beams)
    # step i runs on streams[i % P] with workspace, row pointers and CSR arrays of its own
    streams = [torch.cuda.current_stream(dev)] + [torch.cuda.Stream(dev) for _ in range(P - 1)]
    sp = [C.c_void_p(x.cuda_stream) for x in streams]
    s = sp[0]

    # sizes (outside the timed region)
    st, _, need = m.fspb_plan_create(grid, beams, nb, kern, None, 0)
    wss = [torch.empty(need + 256, dtype=torch.uint8, device=dev) for _ in range(P)]
    wsp = [(w.data_ptr() + 255) // 256 * 256 for w in wss]
    st, h, _ = m.fspb_plan_create(grid, beams, nb, kern, wsp[0], need)
    desc = m.fspb_plan_info(h)
    indptrs = [torch.empty(desc.n_beamlets + 1, dtype=torch.int64, device=dev) for _ in range(P)]
    m.fspb_raytrace(h, s)
    st, nnz = m.fspb_dose_coeffs(h, indptrs[0].data_ptr(), None, None, 0, s)
    m.fspb_plan_destroy(h)
    indices_l = [torch.empty(nnz, dtype=torch.int32, device=dev) for _ in range(P)]
    values_l = [torch.empty(nnz, dtype=torch.float32, device=dev) for _ in range(P)]

    def step(i, timed, P=P):
        q = i % P
        st_, hh, _ = m.fspb_plan_create(grid, beams, nb, kern, wsp[q], need)
        if timed:
            m.fspb_plan_set_timing(hh, 1)
        m.fspb_raytrace(hh, sp[q])
        st_, n_ = m.fspb_dose_coeffs(hh, indptrs[q].data_ptr(), indices_l[q].data_ptr(),
                                     values_l[q].data_ptr(), nnz, sp[q])
        assert st_ == m.FSPB_OK and n_ == nnz
        t = m.fspb_plan_get_timing(hh) if timed else None
        m.fspb_plan_destroy(hh)
        return t

    def timed_steps(P):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(i, False, P)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    for i in range(warmup):
        step(i, False)
    wall = timed_steps(P)
    ms_step_serial = 1e3 * timed_steps(1) / steps if P > 1 else 1e3 * wall / steps

    times = [step(0, True, 1) for _ in range(steps)]
    torch.cuda.synchronize()
    kt = {key: float(np.median([getattr(t, key) for t in times]))
          for key in ("prep_ms", "raytrace_ms", "count_ms", "scan_ms", "fill_ms")}
    fill_s = kt["fill_ms"] * 1e-3
    alg_bytes = 8.0 * nnz                     # FP32 value + int32 column per nonzero
    achieved = alg_bytes / fill_s / 1e9
    workload = fi.CONFIG_NAMES[k]
    out = {
        "workload": workload, "grid": list(prob.grid.shape_xyz), "beams": nb, "beamlets": desc.n_beamlets,
        "nnz": nnz, "plans_in_flight": P, "wall_s": wall,
        "ms_per_step": round(1e3 * wall / steps, 4),
        "ms_per_step_one_stream": round(ms_step_serial, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profile("k_fill", workload),
                     "kernel": "k_fill", "bytes_per_launch": alg_bytes},
        "roofline_alu": valu_roofline(workload, fill_s),
        "kernel_ms": {key: round(v, 4) for key, v in kt.items()},
        # device time of fspb_raytrace + fspb_dose_coeffs (per-kernel medians), as the paper's T_GPU
        "device_ms_per_plan": round(sum(kt.values()), 4),
        "device_nnz_per_s": round(nnz / (sum(kt.values()) * 1e-3), 1),
        "fill_erf_mode": desc.fill_erf_mode,
    }
    csr = (indptrs[0], indices_l[0], values_l[0])
    del indices_l[1:], values_l[1:], wss
    return out, csr, prob


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the rows of D would shard by "
              f"beamlet across GPUs, but only the single-GPU path is implemented.", file=sys.stderr)
        sys.exit(2)
    if args.workload == 3:
        bench_batch(args)
        return
    if args.table1:
        bench_table1(args)
        return
    import torch
    import fspb_inputs as fi

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    head, csr, prob = plan_workload(args.workload, args.steps, args.warmup, args.pipeline)
    nnz = head["nnz"]
    out = {
        "metric": METRIC,
        "value": round(nnz * args.steps / head["wall_s"], 1),
        "unit": "D_ij nonzeros/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": head["workload"], "grid": head["grid"], "beams": head["beams"],
                   "beamlets": head["beamlets"], "nnz": nnz, "plans_in_flight": head["plans_in_flight"]},
        # the same loop on one stream: one plan at a time, nothing overlapped
        "ms_per_step_one_stream": head["ms_per_step_one_stream"],
        "roofline": head["roofline"],
        # the fill against the VALU issue peak (null when the committed counter profile does not
        # match these fill sources or this workload)
        "roofline_alu": head["roofline_alu"],
        "kernel_ms": head["kernel_ms"],
        "device_ms_per_plan": head["device_ms_per_plan"],
        "device_nnz_per_s": head["device_nnz_per_s"],
        "fill_erf_mode": head["fill_erf_mode"],
    }
    n_vox = int(np.prod(prob.grid.shape_xyz))
    n_rows = head["beamlets"]
    if not args.no_cpu_baseline and args.cpu_seconds > 0:
        # the oracle on this host's cores, and the error of the timed plan's CSR against it
        out["cpu_baseline"], out["error_vs_oracle"] = cpu_baseline(prob, args.cpu_seconds, n_rows, csr)
    if not args.no_eq1:
        out["eq1"] = eq1_timings(csr[0], csr[1], csr[2], n_vox, n_rows)
    del csr
    torch.cuda.empty_cache()
    if args.workload == 1 and not args.headline_only:
        # the other two workloads of the metric, measured by the same code
        pel, pcsr, pprob = plan_workload(2, args.steps, args.warmup, args.pipeline)
        pel.pop("wall_s")
        pel["nnz_per_s"] = round(pel["nnz"] / (pel["ms_per_step"] * 1e-3), 1)
        if not args.no_cpu_baseline and args.cpu_seconds > 0:
            pel["error_vs_oracle"] = oracle_error(pprob, pcsr)
        del pcsr
        out["pelvis"] = pel
        torch.cuda.empty_cache()
        out["batch32"] = batch_workload(max(args.steps // 2, 3), 1)[0]
    if not args.no_next:
        out["next_rows"] = next_rows_timings(prob)
    if args.surrogate_epochs is None:                # by default only beside the headline workload
        args.surrogate_epochs = fi.SURROGATE_EPOCHS if args.workload == 1 else 0
    if args.surrogate_epochs > 0:
        out["surrogate"] = surrogate_comparison(args.surrogate_epochs,
                                                cpu=not args.no_cpu_baseline and args.cpu_seconds > 0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
