"""The counter report's arithmetic on the CPU, with synthetic rocprofv3 result
databases: per-kernel averages per dispatch, the calibration of FETCH_SIZE and
WRITE_SIZE on the 1 GiB copy (the copy's bytes divided by what the counter
reads for it), the HBM bytes per launch, and the kernel-source hash."""
import json
import os
import sqlite3

from paper_2604_10357_amd import pmc


def _db(path, counter, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
                "value real)")
    for did, name, val in rows:
        # two partial values per dispatch, as the per-XCD instances of a counter come
        con.execute("insert into counters_collection values (?, ?, ?, ?)", (did, name, counter, val / 2))
        con.execute("insert into counters_collection values (?, ?, ?, ?)", (did, name, counter, val / 2))
    con.commit()
    con.close()


def test_report_calibrates_on_the_copy(tmp_path):
    gib_kib = (1 << 30) / 1024.0
    ns = "void tlfea::(anonymous namespace)::"
    fetch = [(1, ns + "k_elem_rows<RuleT10>(tlfea::AsmArgs, int const*, float*)", 1000.0),
             (2, ns + "k_elem_rows<RuleT10>(tlfea::AsmArgs, int const*, float*)", 3000.0),
             (3, "__amd_rocclr_copyBuffer", gib_kib / 2),  # FETCH_SIZE reads half the copied bytes
             (4, ns + "k_gather_rows<true, true, false>(tlfea::GatherArgs)", 500.0)]
    write = [(1, ns + "k_elem_rows<RuleT10>(tlfea::AsmArgs, int const*, float*)", 4000.0),
             (2, "__amd_rocclr_copyBuffer", gib_kib),
             (3, ns + "k_gather_rows<true, true, false>(tlfea::GatherArgs)", 100.0)]
    _db(str(tmp_path / "fetch" / "a" / "pmc_results.db"), "FETCH_SIZE", fetch)
    _db(str(tmp_path / "write" / "a" / "pmc_results.db"), "WRITE_SIZE", write)
    out = tmp_path / "report.json"
    shape = {"waves": 4, "range_tasks": 768, "range_values": 2048}
    rep = pmc.report(str(tmp_path), str(out), shape)
    assert abs(rep["fetch_size_factor"] - 2.0) < 1e-12 and abs(rep["write_size_factor"] - 1.0) < 1e-12
    rows = rep["kernels"]["k_elem_rows<RuleT10>"]
    assert rows["fetch_size_kib"] == 2000.0                      # mean of the two dispatches
    assert rows["fetch_size_bytes"] == 2000.0 * 1024 * 2.0
    assert rows["write_size_bytes"] == 4000.0 * 1024
    assert rows["hbm_bytes"] == rows["fetch_size_bytes"] + rows["write_size_bytes"]
    g = rep["kernels"]["k_gather_rows<true, true, false>"]
    assert g["hbm_bytes"] == 500.0 * 1024 * 2.0 + 100.0 * 1024
    assert "__amd_rocclr_copyBuffer" not in rep["kernels"]
    assert rep["kernel_source_sha256"] == pmc.kernel_source_hash() and rep["gather_shape"] == shape
    assert json.load(open(out)) == rep
    beam = pmc.report(str(tmp_path), str(tmp_path / "beam.json"), shape, "beam")
    assert beam["workload"].startswith("ancf3243_chain_500000")
