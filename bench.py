"""Benchmark: fused internal force + tangent assembly on one MI355X.

Default workload: the large T10 beam (200 x 20 x 20 Kuhn cells = 480,000
quadratic tetrahedra, 2,022,243 DOF, 169,094,889 CSR values), Mooney-Rivlin +
Kelvin-Voigt, mixed precision, one `tlfea_assemble` call per step (clear f and
the CSR values, then f_int and h * df/dq + df/dqdot with h = 1e-3).  Inputs are
resident in HBM before the timed region.  The FP64 form is timed on the same
mesh for comparison.

Prints one JSON line: metric / value (elements per second, whole call),
roofline of the dominant kernel (algorithmic bytes / its event-timed duration
against 8 TB/s), FP64 comparison, errors against the CPU oracle and the CPU
oracle's own throughput on a bounded sample of the same mesh.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_t10_beam_200x20x20_mixed.json")


def algorithmic_bytes(n_el, n_dof, nnz, n_pn=10, geo_bytes=80):
    """Bytes one fused f + K call must move with this library's data layout:
    K values written once (8 nnz), f written once (8 n_dof), q, qdot and X read
    once (24 n_dof), CSR row offsets (4 n_dof), connectivity (4 n_pn per
    element), reference geometry (80 B per affine element: J0^-1 and det J0) and
    the one-byte node-rank slot map (n_pn^2 per element)."""
    return 8 * nnz + 8 * n_dof + 24 * n_dof + 4 * (n_dof + 1) + n_el * (4 * n_pn + geo_bytes + n_pn * n_pn)


def measured_traffic(precision):
    """HBM bytes per call of the two kernels from the committed counter report
    (FETCH_SIZE / WRITE_SIZE calibrated on a 1 GiB copy), or None when the
    report is missing, is for another precision, or the kernels changed since."""
    if precision != "mixed" or not os.path.exists(TRAFFIC_FILE):
        return None
    from paper_2604_10357_amd import pmc
    with open(TRAFFIC_FILE) as fh:
        rep = json.load(fh)
    if rep.get("kernel_source_sha256") != pmc.kernel_source_hash():
        return None
    ks = rep["kernels"]
    names = [k for k in ks if k.startswith("k_stage_tile<RuleT10, float>") or
             k.startswith("k_gather<RuleT10, float, true, true, false>")]
    if len(names) != 2:
        return None
    return sum(ks[k]["hbm_bytes"] for k in names)


def time_calls(fn, steps, torch):
    s = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(s)
    for _ in range(steps):
        fn()
    end.record(s)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps  # ms


def cpu_baseline(wl, f_gpu, vals_gpu, ro, cols, h, budget_s=12.0):
    """Time the FP64 CPU oracle on a bounded sample (the first elements of the
    mesh, i.e. whole x-slabs) and compare the GPU rows of the nodes whose every
    incident element lies in the sample."""
    import oracle
    from paper_2604_10357_amd import workloads as W

    oracle.build(force=False)
    omat = oracle.material_of(wl.material)
    # calibrate on a small slab, then size the sample to the budget
    n_cal = 2400
    sub = W.Mesh(W.T10, wl.mesh.X, wl.mesh.conn[:n_cal].copy())
    om = oracle.Mesh.of(sub)
    pat = oracle.csr_pattern(om)
    t0 = time.perf_counter()
    oracle.assemble(om, omat, wl.q, wl.qdot, h, 1.0, pattern=pat)
    per_el = (time.perf_counter() - t0) / n_cal
    n = int(min(wl.mesh.n_elem, max(n_cal, budget_s / per_el)))
    n = max(2400, (n // 2400) * 2400)  # whole slabs of 20 x 20 cells
    sub = W.Mesh(W.T10, wl.mesh.X, wl.mesh.conn[:n].copy())
    om = oracle.Mesh.of(sub)
    pat = oracle.csr_pattern(om)
    t0 = time.perf_counter()
    f_ref, v_ref = oracle.assemble(om, omat, wl.q, wl.qdot, h, 1.0, pattern=pat)
    dt = time.perf_counter() - t0
    # nodes all of whose elements are in the sample
    inc_all = np.zeros(wl.mesh.n_coef, dtype=np.int64)
    np.add.at(inc_all, wl.mesh.conn.ravel(), 1)
    inc_sub = np.zeros(wl.mesh.n_coef, dtype=np.int64)
    np.add.at(inc_sub, sub.conn.ravel(), 1)
    inner = np.nonzero((inc_sub == inc_all) & (inc_sub > 0))[0]
    rows = (3 * inner[:, None] + np.arange(3)[None, :]).ravel()
    errs = {}
    ef = np.abs(f_gpu[rows] - f_ref[rows]).max() / np.abs(f_ref[rows]).max()
    ro_s, cols_s = pat
    kd, kmax = 0.0, 0.0
    for r in rows[:: max(1, len(rows) // 3000)]:
        a, b = ro_s[r], ro_s[r + 1]
        ga, gb = ro[r], ro[r + 1]
        assert np.array_equal(cols_s[a:b], cols[ga:gb])
        kd = max(kd, np.abs(vals_gpu[ga:gb] - v_ref[a:b]).max())
        kmax = max(kmax, np.abs(v_ref[a:b]).max())
    errs["f"] = float(ef)
    errs["K"] = float(kd / kmax)
    base = {"value": n / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} of {wl.mesh.n_elem} elements (whole x-slabs), fused f + K, FP64 C oracle, "
                      f"{dt:.1f} s single-threaded"}
    return base, errs, len(rows)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    import torch

    from paper_2604_10357_amd import workloads as W
    from paper_2604_10357_amd.api import TLMesh

    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    wl = W.config5()
    n_el, n_dof = wl.mesh.n_elem, wl.mesh.n_dof
    mesh = TLMesh(wl.mesh, wl.material, args.precision)
    nnz = mesh.build_pattern()
    q = torch.from_numpy(wl.q).cuda()
    qd = torch.from_numpy(wl.qdot).cuda()
    f = torch.empty(n_dof, dtype=torch.float64, device="cuda")
    vals = torch.empty(nnz, dtype=torch.float64, device="cuda")
    h = 1e-3
    torch.cuda.synchronize()
    print(f"[bench] setup {time.perf_counter() - t_setup:.1f} s: {n_el} elements, {n_dof} dof, nnz {nnz}",
          file=sys.stderr, flush=True)

    def step():
        mesh.assemble(q, qd, h, 1.0, f, vals)

    def pass1():
        mesh.assemble_points(q, qd, h, 1.0, True)

    def pass2():
        mesh.assemble_nodes(f, vals)

    for _ in range(args.warmup):
        step()
    ms = time_calls(step, args.steps, torch)
    print(f"[bench] {args.precision}: {ms:.4f} ms per call", file=sys.stderr, flush=True)
    ms1 = time_calls(pass1, args.steps, torch)
    ms2 = time_calls(pass2, args.steps, torch)
    step()  # leave the outputs of a complete call in f / vals
    torch.cuda.synchronize()
    f_h = f.cpu().numpy()
    v_h = vals.cpu().numpy()

    # the hot path is the pair of kernels k_stage_tile (pass 1) + k_gather
    # (pass 2), timed together with events on the stream they run on; its
    # algorithmic bytes are set against the time of the whole call
    B = algorithmic_bytes(n_el, n_dof, nnz)
    achieved = B / (ms * 1e-3) / 1e9
    traffic = measured_traffic(args.precision)
    out = {
        "metric": "f_int+K assembly elements/s and HBM GB/s; mixed vs FP64 at stated error",
        "value": n_el / (ms * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "t10_beam_200x20x20_mr_kv", "elements": n_el, "dof": n_dof, "nnz": nnz,
                   "precision": args.precision, "material": "mooney_rivlin+kelvin_voigt", "h": h},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_stage_tile + k_gather (T10, f + K)", "kernel_ms": ms,
                     "pass1_stage_ms": ms1, "pass2_gather_ms": ms2, "algorithmic_bytes": B},
    }
    ro, cols = mesh.csr_pattern(on_device=False)
    ro, cols = ro.numpy(), cols.numpy()
    if not args.no_fp64 and args.precision == "mixed":
        mesh.set_precision("fp64")
        for _ in range(args.warmup):
            step()
        ms64 = time_calls(step, args.steps, torch)
        ms64_1 = time_calls(pass1, args.steps, torch)
        ms64_2 = time_calls(pass2, args.steps, torch)
        step()
        torch.cuda.synchronize()
        f64, v64 = f.cpu().numpy(), vals.cpu().numpy()
        mesh.set_precision(args.precision)
        out["fp64"] = {"value": n_el / (ms64 * 1e-3), "ms_per_step": ms64, "pass1_stage_ms": ms64_1,
                       "pass2_gather_ms": ms64_2, "achieved_GBs": B / (ms64 * 1e-3) / 1e9,
                       "speedup_mixed_over_fp64": ms64 / ms}
        # mixed against the FP64 GPU result over the whole output
        out["mixed_vs_fp64_gpu"] = {
            "f": float(np.abs(f_h - f64).max() / np.abs(f64).max()),
            "K": float(np.abs(v_h - v64).max() / np.abs(v64).max())}
        print(f"[bench] fp64: {ms64:.4f} ms per call", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        base, errs, nrows = cpu_baseline(wl, f_h, v_h, ro, cols, h)
        out["cpu_baseline"] = base
        out["error_vs_oracle"] = dict(errs, rows=nrows, precision=args.precision, gate=1e-5 if args.precision == "mixed" else 1e-12)
    mesh.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
