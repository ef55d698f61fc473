"""Benchmark: fused internal force + tangent assembly on one MI355X.

Default workload (`--workload t10_beam`): the large T10 beam (200 x 20 x 20
Kuhn cells = 480,000 quadratic tetrahedra, 2,022,243 DOF, 169,094,889 CSR
values), Mooney-Rivlin + Kelvin-Voigt, mixed precision, one `tlfea_assemble`
call per step (f_int and h * df/dq + df/dqdot with h = 1e-3, outputs
overwritten).  Inputs are resident in HBM before the timed region.  The FP64
form is timed on the same mesh for comparison.  Other workloads: `t10_box`
(80 x 8 x 8 cells), `ancf_plate` (256 x 256 ANCF3443 shell, SVK, 3x3x2 rule),
`ancf_beam` (500,000-element ANCF3243 chain, SVK, 3x2x2 rule) and `batched`
(512 T10 cubes in one graph-captured launch pair, against the per-body loop).

Prints one JSON line: metric / value (elements per second, whole call),
roofline of the hot path (algorithmic bytes / its event-timed duration against
8 TB/s, and the counter-measured HBM traffic when it is on record for these
kernels), FP64 comparison, errors against the CPU oracle and the CPU oracle's
own throughput on a bounded sample of the same mesh.
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
FP32_PEAK_TFLOPS = 157.3  # MI355X vector FP32 (dense)
FP64_PEAK_TFLOPS = 78.6


def contraction_flop(wl):
    """FLOPs per element of the tangent contraction alone (the arithmetic floor of
    K_e): per point t_a = A g_a for every (a, i, k) (9 FMA each, 81 n_en) and every
    3x3 block (a, b) from t_a (27 FMA each, 27 n_en^2); constitutive work and f
    not counted."""
    n_en = {1: 10, 2: 16, 3: 8}[wl.mesh.elem_type]
    n_qp = 5 if wl.mesh.elem_type == 1 else int(np.prod(wl.mesh.gl))
    return 2 * n_qp * (81 * n_en + 27 * n_en * n_en)
# committed counter reports: file and the two kernels of the mixed call, per workload
TRAFFIC = {
    "t10_beam": ("hbm_traffic_t10_beam_200x20x20_mixed.json",
                 ("k_elem_rows<RuleT10, false>", "k_gather_rows<true, true, false>")),
    "ancf_beam": ("hbm_traffic_ancf3243_chain_500000_mixed.json",
                  ("k_elem_rows_mc<RuleBeam, true, false>", "k_gather_rows_mc<RuleBeam, true, true, false>")),
}


def algorithmic_bytes(n_el, n_dof, nnz, n_pn=10, geo_bytes=80, extra_per_elem=0, want_k=True):
    """Bytes one fused f + K call must move with this library's data layout:
    K values written once (8 nnz), f written once (8 n_dof), q, qdot and X read
    once (24 n_dof), CSR row offsets (4 n_dof), connectivity (4 n_pn per
    element), reference geometry (80 B per affine element: J0^-1 and det J0;
    per point otherwise), the one-byte node-rank slot map (n_pn^2 per element)
    and per-element scales (ANCF: 16 B)."""
    b = 8 * n_dof + 24 * n_dof + n_el * (4 * n_pn + geo_bytes + extra_per_elem)
    if want_k:
        b += 8 * nnz + 4 * (n_dof + 1) + n_el * n_pn * n_pn
    return b


def method_bytes(wl, nnz):
    """Algorithmic bytes of one fused f + K call, counted on the method's own
    data (the roofline's figure): K values written once (8 nnz), f
    written (8 n_dof), q and qdot read (16 n_dof), connectivity (4 m per element,
    m pattern nodes), reference geometry (80 B per affine T10, 80 B per point for
    ANCF: J0^-1 and det J0) and a 4-byte block slot map (4 n_en^2 per element,
    n_en shape functions).  Config 5: 1,650.9 MB = 3,439 B per element."""
    m = wl.mesh
    if m.elem_type == 1:
        n_pn, geo, n_en = 10, 80, 10
    else:
        n_pn, n_en = m.conn.shape[1], (16 if m.elem_type == 2 else 8)
        geo = 80 * int(np.prod(m.gl)) if m.elem_type == 2 else 80 * 12
    return 8 * nnz + 24 * m.n_dof + m.n_elem * (4 * n_pn + geo + 4 * n_en * n_en)


def mesh_bytes(wl, nnz, affine=True):
    m = wl.mesh
    if m.elem_type == 1:  # T10
        return algorithmic_bytes(m.n_elem, m.n_dof, nnz, 10, 80 if affine else 80 * 5)
    nq = int(np.prod(m.gl))
    return algorithmic_bytes(m.n_elem, m.n_dof, nnz, m.conn.shape[1], 80 if affine else 80 * nq, 16)


def measured_traffic(wname, precision, shape):
    """HBM bytes per call of the two kernels from the workload's committed
    counter report (FETCH_SIZE / WRITE_SIZE calibrated on a 1 GiB copy), or
    None when there is none, or it is for another precision or pass-2 launch
    shape, or the kernels changed since."""
    if precision != "mixed" or wname not in TRAFFIC:
        return None
    fname, kernels = TRAFFIC[wname]
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    from paper_2604_10357_amd import pmc
    with open(path) as fh:
        rep = json.load(fh)
    if rep.get("kernel_source_sha256") != pmc.kernel_source_hash():
        return None
    if rep.get("gather_shape", pmc.DEFAULT_SHAPE) != shape:
        return None
    ks = rep["kernels"]
    if any(k not in ks for k in kernels):
        return None
    return sum(ks[k]["hbm_bytes"] for k in kernels)


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
    mesh) and compare the GPU rows of the nodes whose every incident element
    lies in the sample."""
    import dataclasses

    import oracle

    oracle.build(force=False)
    omat = oracle.material_of(wl.material)
    n_el = wl.mesh.n_elem
    mc = 1 if wl.mesh.elem_type == 1 else 4

    def sample(n):
        sub = dataclasses.replace(wl.mesh, conn=wl.mesh.conn[:n].copy())
        om = oracle.Mesh.of(sub)
        return sub, om, oracle.csr_pattern(om)

    n_cal = min(n_el, 2400)
    sub, om, pat = sample(n_cal)
    t0 = time.perf_counter()
    oracle.assemble(om, omat, wl.q, wl.qdot, h, 1.0, pattern=pat)
    per_el = (time.perf_counter() - t0) / n_cal
    n = int(min(n_el, max(n_cal, budget_s / per_el)))
    sub, om, pat = sample(n)
    t0 = time.perf_counter()
    f_ref, v_ref = oracle.assemble(om, omat, wl.q, wl.qdot, h, 1.0, pattern=pat)
    dt = time.perf_counter() - t0
    # pattern nodes all of whose elements are in the sample
    n_pnodes = int(wl.mesh.conn.max()) + 1
    inc_all = np.bincount(wl.mesh.conn.ravel(), minlength=n_pnodes)
    inc_sub = np.bincount(sub.conn.ravel(), minlength=n_pnodes)
    inner = np.nonzero((inc_sub == inc_all) & (inc_sub > 0))[0]
    coefs = (mc * inner[:, None] + np.arange(mc)[None, :]).ravel()
    rows = (3 * coefs[:, None] + np.arange(3)[None, :]).ravel()
    errs = {}
    ef = np.abs(f_gpu[rows] - f_ref[rows]).max() / np.abs(f_ref[rows]).max()
    ro_s, cols_s = pat
    if n == n_el:
        # the whole mesh: the pattern bit for bit and every value
        errs["pattern_bit_exact"] = bool(np.array_equal(ro_s, ro) and np.array_equal(cols_s, cols))
        kd, kmax = np.abs(vals_gpu - v_ref).max(), np.abs(v_ref).max()
    else:
        # every row of the nodes whose elements all lie in the sample
        lens = ro[rows + 1] - ro[rows]
        assert np.array_equal(lens, ro_s[rows + 1] - ro_s[rows])
        within = np.arange(lens.sum()) - np.repeat(np.cumsum(lens) - lens, lens)
        gi = np.repeat(ro[rows], lens) + within
        si = np.repeat(ro_s[rows], lens) + within
        errs["pattern_bit_exact"] = bool(np.array_equal(cols[gi], cols_s[si]))
        kd, kmax = np.abs(vals_gpu[gi] - v_ref[si]).max(), np.abs(v_ref[si]).max()
    errs["f"] = float(ef)
    errs["K"] = float(kd / kmax)
    cpu = cpu_model()
    base = {"value": n / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} of {n_el} elements, fused f + K, FP64 C oracle, {dt:.1f} s single-threaded",
            "cpu": cpu}
    # the same sample through the oracle's timing-only OpenMP form, all host threads
    t0 = time.perf_counter()
    _, _, threads = oracle.assemble_omp(om, omat, wl.q, wl.qdot, h, 1.0, pat)
    dt_omp = time.perf_counter() - t0
    base_omp = {"value": n / dt_omp, "unit": "elements/s", "cores": threads, "kind": "oracle_openmp",
                "sample": f"first {n} of {n_el} elements, fused f + K, FP64 C oracle with an OpenMP element loop "
                          f"and atomic scatter, {dt_omp:.2f} s on {threads} threads", "cpu": cpu}
    return base, base_omp, errs, len(rows)


def cpu_model():
    """The host CPU's model name and logical CPU count, as the OS reports them."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name} ({os.cpu_count()} logical CPUs)"


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (GB/s, read + write bytes) as the achievable HBM rate."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    ms = time_calls(lambda: b.copy_(a), reps, torch)
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


WORKLOADS = {
    "t10_beam": ("config5", "t10_beam_200x20x20_mr_kv"),
    "t10_box": ("config2", "t10_box_80x8x8_mr_kv"),
    "ancf_plate": ("config3", "ancf3443_plate_256x256_svk"),
    "ancf_beam": ("beam_res32", "ancf3243_chain_500000_svk"),
}


def autotune(args, obj, tune):
    """Pass-2 launch shape: the library's autotuner (run once, before any timed
    call), unless --gather-shape sets one or --no-autotune keeps the default;
    returns what was used."""
    if args.gather_shape:
        obj.set_gather_shape(*args.gather_shape)
        return {"autotuned": False, "gather_shape": obj.gather_shape()[0]}
    if args.no_autotune:
        return {"autotuned": False, "gather_shape": obj.gather_shape()[0]}
    t0 = time.perf_counter()
    shape, ms, _, _ = tune()
    out = {"autotuned": True, "gather_shape": shape, "tuned_ms_per_call": ms,
           "autotune_s": time.perf_counter() - t0}
    print(f"[bench] autotuned pass-2 shape {shape} ({ms:.3f} ms per call)", file=sys.stderr, flush=True)
    return out


def bench_mesh(args, torch, wl, wname):
    from paper_2604_10357_amd.api import TLMesh

    t_setup = time.perf_counter()
    n_el, n_dof = wl.mesh.n_elem, wl.mesh.n_dof
    mesh = TLMesh(wl.mesh, wl.material, args.precision)
    nnz = mesh.build_pattern()
    q = torch.from_numpy(wl.q).cuda()
    qd = torch.from_numpy(wl.qdot).cuda()
    f = torch.empty(n_dof, dtype=torch.float64, device="cuda")
    vals = torch.empty(nnz, dtype=torch.float64, device="cuda")
    h = 1e-3
    torch.cuda.synchronize()
    print(f"[bench] {wname} setup {time.perf_counter() - t_setup:.1f} s: {n_el} elements, {n_dof} dof, nnz {nnz}",
          file=sys.stderr, flush=True)
    tuning = autotune(args, mesh, lambda: mesh.autotune(q, qd, h, f, vals, reps=5))

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

    # the hot path is the pair of kernels of one call (pass 1 + pass 2), timed
    # together with events on the stream they run on; the method's algorithmic
    # bytes are set against the time of the whole call, the library's own count
    # of what its data layout must move beside them
    B = method_bytes(wl, nnz)
    B_layout = mesh_bytes(wl, nnz)
    achieved = B / (ms * 1e-3) / 1e9
    traffic = measured_traffic(wname, args.precision, tuning["gather_shape"])
    kname = {1: "T10", 2: "ANCF3443", 3: "ANCF3243"}[wl.mesh.elem_type]
    # the tangent in mixed precision takes the element-row kernels
    rows_path = args.precision == "mixed" and os.environ.get("TLFEA_ELEMENT_ROWS") != "0"
    mat = "mooney_rivlin" if wl.material.kind == 2 else "svk"
    if wl.material.kv_eta or wl.material.kv_lambda:
        mat += "+kelvin_voigt"
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
        "config": {"workload": WORKLOADS[wname][1], "elements": n_el, "dof": n_dof, "nnz": nnz,
                   "precision": args.precision, "material": mat, "h": h},
        "tuning": tuning,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": (f"k_elem_rows{'' if kname == 'T10' else '_mc'} + k_gather_rows"
                                f"{'' if kname == 'T10' else '_mc'} ({kname}, f + K)" if rows_path else
                                f"k_stage_tile + k_gather ({kname}, f + K)"), "kernel_ms": ms,
                     "pass1_stage_ms": ms1, "pass2_gather_ms": ms2, "algorithmic_bytes": B,
                     "algorithmic_bytes_layout": B_layout,
                     "frac_layout": B_layout / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        # the same call against the vector arithmetic roofline (contraction FLOPs only)
        # the shell's mixed contraction runs on the matrix cores (FP32 MFMA, the same 157.3 peak)
        "valu": {"units": ("matrix cores (fp32 MFMA 16x16x4)" if kname == "ANCF3443" and rows_path
                           else "vector ALUs"),
                 "flop_per_element": contraction_flop(wl),
                 "achieved_TFLOPs": contraction_flop(wl) * n_el / (ms * 1e-3) / 1e12,
                 "peak_TFLOPs": FP32_PEAK_TFLOPS if args.precision == "mixed" else FP64_PEAK_TFLOPS,
                 "frac": contraction_flop(wl) * n_el / (ms * 1e-3) / 1e12
                 / (FP32_PEAK_TFLOPS if args.precision == "mixed" else FP64_PEAK_TFLOPS)},
    }
    # Newton step pieces on the same mesh: H = M/h + h K_t (one call, the
    # mass term inside pass 2) and the gradient M (v - v_prev)/h + f_int;
    # density: the paper's scaling benchmarks use 2700 kg/m^3
    rho = 2700.0
    mesh.build_mass(rho)
    fn = torch.empty_like(f)
    hn = torch.empty_like(vals)
    g = torch.empty_like(f)
    vp = torch.zeros_like(qd)
    mesh.assemble_newton(q, qd, h, fn, hn)
    ms_newton = time_calls(lambda: mesh.assemble_newton(q, qd, h, fn, hn), args.steps, torch)
    mesh.newton_gradient(qd, vp, fn, None, h, g)
    ms_grad = time_calls(lambda: mesh.newton_gradient(qd, vp, fn, None, h, g), args.steps, torch)
    mc = 1 if wl.mesh.elem_type == 1 else 4  # coefficient vectors per node
    n_pairs = nnz // (9 * mc * mc)  # adjacent node pairs (one 3 mc x 3 mc block each)
    # mass blocks + neighbour ids; v, v_prev, f_int read, g written
    grad_bytes = (8 * mc * mc + 4) * n_pairs + 8 * n_dof * 4
    out["newton"] = {"assemble_newton_ms": ms_newton, "vs_assemble": ms_newton / ms, "gradient_ms": ms_grad,
                     "gradient_GBs": grad_bytes / (ms_grad * 1e-3) / 1e9, "gradient_bytes": grad_bytes,
                     "density": rho}
    print(f"[bench] newton matrix {ms_newton:.4f} ms, gradient {ms_grad:.4f} ms", file=sys.stderr, flush=True)
    # the first-order inner solver: 100 AdamW iterations (f_int + gradient +
    # update), checked every 25 (graph replays in between)
    ms_fint = time_calls(lambda: mesh.internal_force(q, qd, fn), args.steps, torch)
    s_ad = torch.cuda.Stream()
    s_ad.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s_ad):
        work = torch.empty(4 * n_dof, dtype=torch.float64, device="cuda")
        vv = qd.clone()
        qq = torch.empty_like(q)
        mesh.adamw_solve(q, qd, vv, h, 1e-4, max_iters=26, check_every=25, q=qq, work=work)
        vv.copy_(qd)
        s_ad.synchronize()
        t0 = time.perf_counter()
        _, _, iters, _, _ = mesh.adamw_solve(q, qd, vv, h, 1e-4, max_iters=101, check_every=25, q=qq,
                                             work=work)
        s_ad.synchronize()
        dt = time.perf_counter() - t0
    out["adamw"] = {"iterations": iters, "ms_per_iteration": dt * 1e3 / iters, "internal_force_ms": ms_fint,
                    "check_every": 25}
    print(f"[bench] adamw {dt * 1e3 / iters:.4f} ms per inner iteration (f_int alone {ms_fint:.4f} ms)",
          file=sys.stderr, flush=True)
    del work
    if not (wl.material.kv_eta or wl.material.kv_lambda):
        # symmetric tangent: the upper triangle alone (half the matrix writes)
        nnz_u = mesh.build_upper_pattern()
        vu = torch.empty(nnz_u, dtype=torch.float64, device="cuda")
        mesh.assemble_upper(q, qd, h, 1.0, f, vu)
        ms_u = time_calls(lambda: mesh.assemble_upper(q, qd, h, 1.0, f, vu), args.steps, torch)
        # the Newton matrix M/h + h K in the same storage (the mass is built above)
        mesh.assemble_newton_upper(q, qd, h, f, vu)
        ms_nu = time_calls(lambda: mesh.assemble_newton_upper(q, qd, h, f, vu), args.steps, torch)
        out["upper"] = {"ms_per_step": ms_u, "vs_full": ms_u / ms, "nnz_upper": nnz_u,
                        "newton_upper_ms": ms_nu}
        print(f"[bench] upper triangle {ms_u:.4f} ms, Newton matrix upper {ms_nu:.4f} ms", file=sys.stderr,
              flush=True)
        del vu
    ro, cols = mesh.csr_pattern(on_device=False)
    ro, cols = ro.numpy(), cols.numpy()
    if not args.no_fp64 and args.precision == "mixed":
        mesh.set_precision("fp64")
        # the FP64 kernels get a launch shape of their own
        tuning64 = autotune(args, mesh, lambda: mesh.autotune(q, qd, h, f, vals, reps=5))
        for _ in range(args.warmup):
            step()
        ms64 = time_calls(step, args.steps, torch)
        ms64_1 = time_calls(pass1, args.steps, torch)
        ms64_2 = time_calls(pass2, args.steps, torch)
        step()
        torch.cuda.synchronize()
        f64, v64 = f.cpu().numpy(), vals.cpu().numpy()
        mesh.set_precision(args.precision)
        mesh.set_gather_shape(*[tuning["gather_shape"][k] for k in ("waves", "range_tasks", "range_values")])
        out["fp64"] = {"value": n_el / (ms64 * 1e-3), "ms_per_step": ms64, "tuning": tuning64, "pass1_stage_ms": ms64_1,
                       "pass2_gather_ms": ms64_2, "achieved_GBs": B / (ms64 * 1e-3) / 1e9,
                       "frac": B / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "valu_frac_fp64": contraction_flop(wl) * n_el / (ms64 * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                       "speedup_mixed_over_fp64": ms64 / ms}
        # mixed against the FP64 GPU result over the whole output
        out["mixed_vs_fp64_gpu"] = {
            "f": float(np.abs(f_h - f64).max() / np.abs(f64).max()),
            "K": float(np.abs(v_h - v64).max() / np.abs(v64).max())}
        print(f"[bench] fp64: {ms64:.4f} ms per call", file=sys.stderr, flush=True)
    if wname == "t10_beam":
        # context: the backward product on the same mesh, and a plain device copy
        w = torch.from_numpy(wl.w).cuda() if wl.w is not None else torch.ones_like(q)
        # the product the method's differentiation asks for (positions and material
        # constants), and the full one with the velocity product too
        mesh.vjp(q, qd, w, want_qdot=False)
        out["vjp_ms"] = time_calls(lambda: mesh.vjp(q, qd, w, want_qdot=False), max(3, args.steps // 4), torch)
        mesh.vjp(q, qd, w)
        out["vjp_with_qdot_ms"] = time_calls(lambda: mesh.vjp(q, qd, w), max(3, args.steps // 4), torch)
        out["copy_GBs"] = copy_bandwidth(torch)
    if wname == "t10_beam" and not args.no_batched:
        # the batched form on the 512 cubes of the batched workload, same precision
        del f, vals, fn, hn, g
        torch.cuda.empty_cache()
        bo = bench_batched(args, torch)
        out["batched"] = {"workload": bo["config"]["workload"], "bodies": bo["config"]["bodies"],
                          "elements": bo["config"]["elements"], "nnz": bo["config"]["nnz"],
                          "graph_ms": bo["ms_per_step"], "loop_ms": bo["per_body_loop"]["ms_per_step"],
                          "speedup_graph_over_loop": bo["per_body_loop"]["speedup_batched_over_loop"],
                          "elements_per_s": bo["value"], "achieved_GBs": bo["roofline"]["achieved"],
                          "frac": bo["roofline"]["frac"], "algorithmic_bytes": bo["roofline"]["algorithmic_bytes"],
                          "kernel": bo["roofline"]["kernel"], "tuning": bo["tuning"]}
        if "fp64" in bo:
            out["batched"]["fp64"] = bo["fp64"]
        print(f"[bench] batched: graph {bo['ms_per_step']:.3f} ms, loop {bo['per_body_loop']['ms_per_step']:.3f} ms",
              file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        base, base_omp, errs, nrows = cpu_baseline(wl, f_h, v_h, ro, cols, h)
        out["cpu_baseline"] = base
        out["cpu_baseline_openmp"] = base_omp
        out["error_vs_oracle"] = dict(errs, rows=nrows, precision=args.precision,
                                      gate=1e-5 if args.precision == "mixed" else 1e-12)
    mesh.close()
    return out


def bench_batched(args, torch):
    """Config-4 style batch: 512 T10 cubes, one graph-captured launch pair vs a
    loop of per-body calls."""
    from paper_2604_10357_amd import workloads as W
    from paper_2604_10357_amd.api import TLBatch, TLMesh

    wls = W.config4()
    meshes = []
    for wl in wls:
        m = TLMesh(wl.mesh, wl.material, args.precision)
        m.build_pattern()
        meshes.append(m)
    b = TLBatch(meshes)
    q = torch.from_numpy(np.concatenate([wl.q for wl in wls])).cuda()
    qd = torch.from_numpy(np.concatenate([wl.qdot for wl in wls])).cuda()
    hs = torch.full((len(wls),), 1e-3, dtype=torch.float64, device="cuda")
    nd, nz = b.dof_off[-1], b.nnz_off[-1]
    f = torch.empty(nd, dtype=torch.float64, device="cuda")
    vals = torch.empty(nz, dtype=torch.float64, device="cuda")
    n_el = sum(wl.mesh.n_elem for wl in wls)
    B = sum(method_bytes(wl, m.nnz) for wl, m in zip(wls, meshes))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tuning = autotune(args, b, lambda: b.autotune(q, qd, hs, f, vals, reps=5))
        tuning["schedule"] = b.schedule()
        for _ in range(args.warmup):
            b.assemble(q, qd, hs, f, vals)
        ms = time_calls(lambda: b.assemble(q, qd, hs, f, vals), args.steps, torch)
        # every schedule at the tuned shape, for the record
        kept = b.schedule()
        sched_ms = {}
        for name, pers, te in (("per_item", False, 25), ("persistent_lpt_25", True, 25), ("persistent_lpt_16", True, 16)):
            if pers and args.precision != "mixed":
                continue
            b.set_schedule(pers, te)
            for _ in range(args.warmup):
                b.assemble(q, qd, hs, f, vals)
            sched_ms[name] = time_calls(lambda: b.assemble(q, qd, hs, f, vals), args.steps, torch)
        b.set_schedule(bool(kept["persistent"]), kept["tile_elems"])
        tuning["schedules_ms"] = sched_ms
        for _ in range(args.warmup):
            b.assemble(q, qd, hs, f, vals, loop=True)
        ms_loop = time_calls(lambda: b.assemble(q, qd, hs, f, vals, loop=True), args.steps, torch)
    s.synchronize()
    fp64 = None
    if args.precision == "mixed":
        # the plain FP64 form of the same batch, and the mixed result against it
        f_mx, v_mx = f.cpu().numpy(), vals.cpu().numpy()
        meshes64 = []
        for wl in wls:
            m = TLMesh(wl.mesh, wl.material, "fp64")
            m.build_pattern()
            meshes64.append(m)
        b64 = TLBatch(meshes64)
        with torch.cuda.stream(s):
            for _ in range(args.warmup):
                b64.assemble(q, qd, hs, f, vals)
            ms64 = time_calls(lambda: b64.assemble(q, qd, hs, f, vals), args.steps, torch)
            b64.assemble(q, qd, hs, f, vals)
        s.synchronize()
        f64, v64 = f.cpu().numpy(), vals.cpu().numpy()
        fp64 = {"ms_per_step": ms64, "value": n_el / (ms64 * 1e-3), "speedup_mixed_over_fp64": ms64 / ms,
                "mixed_vs_fp64": {"f": float(np.abs(f_mx - f64).max() / np.abs(f64).max()),
                                  "K": float(np.abs(v_mx - v64).max() / np.abs(v64).max())},
                "kernel": "k_stage_batch + k_gather_batch (one graph)"}
        b64.close()
        for m in meshes64:
            m.close()
    achieved = B / (ms * 1e-3) / 1e9
    out = {
        "metric": "f_int+K assembly elements/s and HBM GB/s; mixed vs FP64 at stated error",
        "value": n_el / (ms * 1e-3), "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": "t10_cubes_x512_batched", "bodies": len(wls), "elements": n_el, "dof": int(nd),
                   "nnz": int(nz), "precision": args.precision},
        "tuning": tuning,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": (("k_elem_rows_batch_lpt + k_gather_rows_batch_lpt (persistent, one graph)"
                                 if tuning["schedule"]["persistent"] else
                                 "k_elem_rows_batch + k_gather_rows_batch (one graph)") if args.precision == "mixed"
                                else "k_stage_batch + k_gather_batch (one graph)"), "kernel_ms": ms,
                     "algorithmic_bytes": B},
        "per_body_loop": {"ms_per_step": ms_loop, "value": n_el / (ms_loop * 1e-3),
                          "speedup_batched_over_loop": ms_loop / ms},
    }
    if fp64 is not None:
        out["fp64"] = fp64
    b.close()
    for m in meshes:
        m.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--workload", default="t10_beam", choices=list(WORKLOADS) + ["batched"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-cube batched leg of the default run")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--gather-shape", type=int, nargs=3, metavar=("WAVES", "RANGE_TASKS", "RANGE_VALUES"))
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    import torch

    from paper_2604_10357_amd import workloads as W

    torch.cuda.set_device(0)
    if args.workload == "batched":
        out = bench_batched(args, torch)
    else:
        wl = getattr(W, WORKLOADS[args.workload][0])()
        out = bench_mesh(args, torch, wl, args.workload)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
