"""Hardware-counter workload and HBM-traffic report for the assembly kernels.

Run under ``rocprofv3 --pmc``, once per counter (FETCH_SIZE, then WRITE_SIZE):

    rocprofv3 --pmc FETCH_SIZE -d <dir>/fetch -o pmc -- python3 -m paper_2604_10357_amd.pmc run [MESH] [W T V]
    rocprofv3 --pmc WRITE_SIZE -d <dir>/write -o pmc -- python3 -m paper_2604_10357_amd.pmc run [MESH] [W T V]
    python3 -m paper_2604_10357_amd.pmc report <dir> <out.json> [MESH] [W T V]

MESH is `t10` (default: the 480,000-element T10 beam, Mooney-Rivlin +
Kelvin-Voigt) or `beam` (the 500,000-element ANCF3243 chain, SVK); W T V is the
pass-2 launch shape (waves, range_tasks, range_values) the assemblies use;
without it, the default shape of the T10 beam.

The workload assembles the mesh (mixed precision) three times and copies a
1 GiB device buffer twice.  The copy has known traffic (1 GiB read, 1 GiB written) and calibrates
each counter: FETCH_SIZE and WRITE_SIZE are scaled by 1 GiB divided by what
they report for the copy.  The report stores, per kernel, the average
counter values per dispatch, the calibrated HBM bytes per launch, and the
SHA-256 of the kernel sources so that a later change of the kernels can be
detected (the benchmark then reports the traffic as unknown).
"""
from __future__ import annotations

import glob
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/assemble.hip", "csrc/kernel_common.h", "csrc/material.h", "csrc/rules.h",
                  "csrc/tables.h", "csrc/tlfea_internal.h"]
COPY_BYTES = 1 << 30


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(rel.encode())
            h.update(fh.read())
    return h.hexdigest()


DEFAULT_SHAPE = {"waves": 4, "range_tasks": 768, "range_values": 2048}  # T10 built in mixed precision


MESHES = {"t10": ("config5", "t10_beam_200x20x20_mr_kv mixed"),
          "beam": ("beam_res32", "ancf3243_chain_500000_svk mixed")}


def _shape(args) -> dict:
    if not args:
        return dict(DEFAULT_SHAPE)
    w, t, v = (int(x) for x in args)
    return {"waves": w, "range_tasks": t, "range_values": v}


def _mesh_and_shape(args):
    mesh = "t10"
    if args and args[0] in MESHES:
        mesh, args = args[0], args[1:]
    return mesh, _shape(args)


def run(shape: dict, mesh: str = "t10") -> None:
    import torch

    from . import workloads as W
    from .api import TLMesh

    wl = getattr(W, MESHES[mesh][0])()
    m = TLMesh(wl.mesh, wl.material, "mixed")
    m.build_pattern()
    m.set_gather_shape(shape["waves"], shape["range_tasks"], shape["range_values"])
    q = torch.from_numpy(wl.q).cuda()
    qd = torch.from_numpy(wl.qdot).cuda()
    f = torch.empty(m.n_dof, dtype=torch.float64, device="cuda")
    v = torch.empty(m.nnz, dtype=torch.float64, device="cuda")
    for _ in range(3):
        m.assemble(q, qd, 1e-3, 1.0, f, v)
    a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    m.close()
    print("pmc workload done", flush=True)


def _per_kernel(db_dir: str, counter: str) -> dict:
    """{short kernel name: [value per dispatch]} for one counter."""
    out: dict = {}
    for f in glob.glob(os.path.join(db_dir, "**", "*_results.db"), recursive=True):
        cur = sqlite3.connect(f).cursor()
        q = ("select dispatch_id, kernel_name, sum(value) from counters_collection "
             "where counter_name = ? group by dispatch_id")
        for _, kname, val in cur.execute(q, (counter,)):
            short = kname.replace("tlfea::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
            out.setdefault(short, []).append(float(val))
    return out


def report(base: str, out_json: str, shape: dict, mesh: str = "t10") -> dict:
    res = {"workload": MESHES[mesh][1], "gather_shape": shape,
           "kernel_source_sha256": kernel_source_hash(), "copy_bytes": COPY_BYTES, "kernels": {}}
    for counter, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        per = _per_kernel(os.path.join(base, sub), counter)
        copy = max(per.get("__amd_rocclr_copyBuffer", [0.0]))
        if copy <= 0:
            raise RuntimeError(f"no copy dispatch found for {counter}")
        factor = COPY_BYTES / (copy * 1024.0)
        res[counter.lower() + "_factor"] = factor
        for k, vals in per.items():
            if not (k.startswith("k_stage") or k.startswith("k_gather") or k.startswith("k_elem")):
                continue
            mean_kib = sum(vals) / len(vals)
            e = res["kernels"].setdefault(k, {})
            e[counter.lower() + "_kib"] = mean_kib
            e[counter.lower() + "_bytes"] = mean_kib * 1024.0 * factor
    for e in res["kernels"].values():
        e["hbm_bytes"] = e.get("fetch_size_bytes", 0.0) + e.get("write_size_bytes", 0.0)
    with open(out_json, "w") as fh:
        json.dump(res, fh, indent=1)
    return res


if __name__ == "__main__":
    if len(sys.argv) in (2, 3, 5, 6) and sys.argv[1] == "run":
        mesh, shape = _mesh_and_shape(sys.argv[2:])
        run(shape, mesh)
    elif len(sys.argv) in (4, 5, 7, 8) and sys.argv[1] == "report":
        mesh, shape = _mesh_and_shape(sys.argv[4:])
        print(json.dumps(report(sys.argv[2], sys.argv[3], shape, mesh), indent=1))
    else:
        print(__doc__)
        sys.exit(2)
