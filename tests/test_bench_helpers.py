"""CPU checks of bench.py's host-side helpers: the algorithmic work model, the roofline choice,
the counter summary and its plan / source checks, and the equal-error interpolation."""
import json

import pytest

import bench


def test_algorithmic_work_counts():
    T, nlat, M, K = 255, 384, 4, 4
    w = bench.algorithmic_work(T, nlat, M, K, 1, "fp64")
    ncoef = (T + 1) * (T + 2) // 2
    states = 1 + (K - 1) * M                                      # f_E evaluations per step
    assert w["synthesis"][0] == pytest.approx(6 * 2.0 * ncoef * nlat * states)
    assert w["analysis"][0] == pytest.approx(7 * 2.0 * ncoef * nlat * states)
    tables = 2.0 * ncoef * (nlat // 2) * 8 * K                    # both tables once per launch
    assert w["synthesis"][1] > tables and w["analysis"][1] > tables
    w32 = bench.algorithmic_work(T, nlat, M, K, 1, "fp32")
    for k in ("synthesis", "analysis", "grid"):
        assert w32[k][1] < w[k][1]                                # FP32 tables and columns
    assert w32["update"] == w["update"]                           # the update stays FP64
    # batch scales the per-state terms, not the tables
    w4 = bench.algorithmic_work(T, nlat, M, K, 4, "fp64")
    assert w4["synthesis"][0] == pytest.approx(4 * w["synthesis"][0])
    assert w4["synthesis"][1] < 4 * w["synthesis"][1]
    # fused update: the tendencies (written by the analysis, read M times per sweep by the update)
    # leave the count; every other byte moves from the update class to the analysis
    wf = bench.algorithmic_work(T, nlat, M, K, 1, "fp64", fused=True)
    e_bytes = 16.0 * ncoef * (3 * states + 3 * M * K)
    assert wf["analysis"][1] + wf["update"][1] == pytest.approx(w["analysis"][1] + w["update"][1] - e_bytes)
    assert wf["update"][1] == 0.0                                 # no update-class launch left
    assert bench.algorithmic_work(T, nlat, M, K, 1, "fp64", True, True)["update"][1] == 0.0
    assert wf["synthesis"] == w["synthesis"] and wf["grid"] == w["grid"]
    # the dominant kernel of the headline step by hand, per launch (4 launches, 13/4 states each):
    # both tables once, 5 Fourier fields per state, the node update's state I/O
    # (K-1)(3+5M) + (6+2M) complex per coefficient spread over the launches
    per_launch = (2 * ncoef * (nlat // 2) * 8 + 13 / 4 * 5 * 16 * nlat * (T + 1)
                  + 16 * ncoef * ((K - 1) * (3 + 5 * M) + (6 + 2 * M)) / 4)
    assert wf["analysis"][1] / K == pytest.approx(per_launch)
    assert per_launch == pytest.approx(137.537024e6)
    # regenerated synthesis tables: same flops, the table bytes replaced by the small recurrence data
    wr = bench.algorithmic_work(T, nlat, M, K, 1, "fp64", syn_recur=True)
    assert wr["synthesis"][0] == w["synthesis"][0]
    assert w["synthesis"][1] - wr["synthesis"][1] > 0.9 * tables
    assert wr["analysis"] == w["analysis"]
    # restarting analysis: a quarter of the table bytes per launch
    wa = bench.algorithmic_work(T, nlat, M, K, 1, "fp64", ana_recur=True)
    assert w["analysis"][1] - wa["analysis"][1] == pytest.approx(0.75 * tables)
    # the first launch's own plan: only its launch changes
    w1 = bench.algorithmic_work(T, nlat, M, K, 1, "fp64", syn_recur1=True, ana_recur1=True)
    per = tables / K
    nhp = (nlat // 2 + 15) // 16 * 16
    rec = 32.0 * (T + 1) * (T + 16) + 8.0 * (T + 1) * nhp
    assert w["synthesis"][1] - w1["synthesis"][1] == pytest.approx(per - rec)
    assert w["analysis"][1] - w1["analysis"][1] == pytest.approx(0.75 * per)


def test_roofline_entry_picks_the_smaller_ceiling():
    # AI = 1 flop/B: bandwidth-bound at 8 TB/s
    e = bench.roofline_entry(1e9, 1e9, 1e-3, 1, "fp64")
    assert e["bound"] == "hbm" and e["unit"] == "GB/s"
    assert e["achieved"] == pytest.approx(1000.0)
    assert e["frac"] == pytest.approx(1000.0 / bench.PEAK_HBM_GBS, rel=1e-3)
    # AI = 1000 flop/B: MFMA-bound
    e = bench.roofline_entry(1e12, 1e9, 1e-1, 1, "fp64")
    assert e["bound"] == "mfma" and e["unit"] == "TFLOP/s"
    assert e["achieved"] == pytest.approx(10.0)


def _csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Kernel_Name,Counter_Name,Counter_Value\n")
        for name, v in rows:
            f.write(f'"{name}",{counter},{v}\n')


def test_summarize_pmc_scales_by_the_copy_and_uses_the_tuned_variant(tmp_path):
    plan = {"syn_lat_tiles": 2, "syn_depth": 2, "ana_depth": 2, "ana_interleave": 1, "fuse_update": 1,
            "syn_recur": 0, "ana_recur": 0}
    logs = []
    for name in ("f.log", "w.log"):
        p = tmp_path / name
        p.write_text("rocprof noise\n" + json.dumps({"metric": "m", "legendre_plan": plan}) + "\n")
        logs.append(str(p))
    copy_kib = 256 * 1024 / 2.0                                   # counter reads half the bytes
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [
        ("__amd_rocclr_copyBuffer(...)", copy_kib),
        ("void k_synthesis<0, double, 2, 2, false, false>(double const*)", 1000.0),
        ("void k_synthesis<0, double, 2, 2, false, false>(double const*)", 3000.0),
        ("void k_synthesis<0, double, 2, 2, false, true>(double const*)", 2000.0),   # first launch
        ("void k_synthesis<0, double, 1, 8, false, false>(double const*)", 99999.0),  # an autotuner trial
        ("void k_synthesis<0, double, 2, 2, true, false>(double const*)", 77777.0),   # regenerating trial
        ("void k_analysis_swe<0, double, 2, false>(double const*)", 500.0),
        ("void k_analysis_swe<0, double, 2, true>(double const*)", 88888.0),     # regenerating trial
        ("void k_grid_swe<768, double>(x)", 10.0),
        ("void k_update<4>(UpdateArgs)", 20.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [
        ("__amd_rocclr_copyBuffer(...)", 256 * 1024.0),
        ("void k_synthesis<0, double, 2, 2, false, false>(double const*)", 100.0),
        ("void k_synthesis<0, double, 2, 2, false, true>(double const*)", 100.0),
        ("void k_analysis_swe<0, double, 2, false>(double const*)", 50.0),
        ("void k_grid_swe<768, double>(x)", 40.0),
        ("void k_update<4>(UpdateArgs)", 30.0)])
    out = tmp_path / "t.json"
    bench.summarize_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 256, str(out), logs)
    t = json.loads(out.read_text())
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    syn = t["kernels"]["synthesis"]
    assert syn["kernel_name"] == ("void k_synthesis<0, double, 2, 2, false, false> + "
                                  "void k_synthesis<0, double, 2, 2, false, true>")
    assert syn["dispatches"] == 3
    assert syn["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert syn["write_bytes_per_launch"] == pytest.approx(100.0 * 1024)
    assert set(t["kernels"]) == {"synthesis", "analysis", "grid", "update"}
    assert t["kernels"]["analysis"]["fetch_bytes_per_launch"] == pytest.approx(500.0 * 1024 * 2.0)
    assert t["legendre_plan"] == plan


def test_summarize_pmc_counts_both_launch_shapes(tmp_path):
    """Streamed tables for the node launches, regenerating variants for the first f_E (one state
    per member): both kernels of each class are averaged, autotuner trials of other variants and
    adjoint kernels are not."""
    plan = {"syn_lat_tiles": 2, "syn_depth": 2, "ana_depth": 2, "ana_interleave": 1, "fuse_update": 1,
            "syn_recur": 0, "ana_recur": 0}
    plan1 = dict(plan, syn_lat_tiles=4, syn_recur=1, ana_recur=1)
    logs = []
    for name in ("f.log", "w.log"):
        p = tmp_path / name
        p.write_text(json.dumps({"metric": "m", "legendre_plan": plan,
                                 "legendre_plan_one_state": plan1}) + "\n")
        logs.append(str(p))
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [
        ("__amd_rocclr_copyBuffer(...)", 256 * 1024.0),
        ("void k_synthesis<0, double, 2, 2, false, false>(double const*)", 1000.0),
        ("void k_synthesis<0, double, 4, 2, true, true>(double const*)", 200.0),     # first launch
        ("void k_synthesis<0, double, 4, 2, true, false>(double const*)", 55555.0),  # trial
        ("void k_analysis_swe<0, double, 2, false>(double const*)", 400.0),
        ("void k_analysis_swe<0, double, 2, true>(double const*)", 100.0),           # first launch
        ("void k_analysis_swe<0, double, 4, true>(double const*)", 66666.0),         # trial
        ("k_prep_cml_adj(double const*, int, double*, bool)", 44444.0)])             # adjoint
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [
        ("__amd_rocclr_copyBuffer(...)", 256 * 1024.0),
        ("void k_synthesis<0, double, 2, 2, false, false>(double const*)", 10.0),
        ("void k_analysis_swe<0, double, 2, false>(double const*)", 20.0)])
    out = tmp_path / "t.json"
    bench.summarize_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 256, str(out), logs)
    t = json.loads(out.read_text())
    assert t["kernels"]["synthesis"]["dispatches"] == 2
    assert t["kernels"]["synthesis"]["fetch_bytes_per_launch"] == pytest.approx(600.0 * 1024)
    assert t["kernels"]["analysis"]["fetch_bytes_per_launch"] == pytest.approx(250.0 * 1024)
    assert "update" not in t["kernels"]
    assert t["legendre_plan_one_state"] == plan1


def test_summarize_pmc_rejects_runs_with_different_variants(tmp_path):
    logs = []
    for name, d in (("f.log", 2), ("w.log", 4)):
        p = tmp_path / name
        p.write_text(json.dumps({"metric": "m", "legendre_plan": {"syn_lat_tiles": 2, "syn_depth": d,
                                                                  "ana_depth": 2, "ana_interleave": 1}}))
        logs.append(str(p))
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer(...)", 1.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer(...)", 1.0)])
    with pytest.raises(RuntimeError):
        bench.summarize_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 256,
                            str(tmp_path / "t.json"), logs)


def test_traffic_is_reported_only_for_the_profiled_sources_and_plan(tmp_path, monkeypatch):
    plan = {"syn_lat_tiles": 2, "syn_depth": 2, "ana_depth": 2, "ana_interleave": 1}
    t = {"source_sha": bench.source_hash(), "legendre_plan": plan,
         "kernels": {k: {"fetch_bytes_per_launch": 1.0, "write_bytes_per_launch": 2.0}
                     for k in ("synthesis", "analysis", "grid", "update")}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.traffic_for("analysis", plan) == 3.0
    other = dict(plan, syn_depth=4)
    assert bench.traffic_for("synthesis", other) is None           # another synthesis variant
    assert bench.traffic_for("analysis", other) == 3.0             # the analysis is unchanged
    assert bench.traffic_for("grid", other) == 3.0                 # grid does not depend on it
    assert bench.traffic_for("analysis", dict(plan, ana_depth=4)) is None
    assert bench.traffic_for("analysis", plan, plan) == 3.0          # no separate one-state plan
    assert bench.traffic_for("analysis", plan, dict(plan, ana_recur=1)) is None
    t["source_sha"] = "0" * 16
    f.write_text(json.dumps(t))
    assert bench.traffic_for("grid", plan) is None                 # other kernel sources


def test_speedup_at_equal_error_interpolates_log_log():
    rows = [{"method": "IMEX-o2", "dt": 2.0, "seconds": 1.0, "error": 1e-6},
            {"method": "IMEX-o2", "dt": 1.0, "seconds": 2.0, "error": 1e-7},
            {"method": "dSDC", "dt": 100.0, "seconds": 0.5, "error": 10 ** -6.5},   # half way
            {"method": "dSDC", "dt": 200.0, "seconds": 0.1, "error": 1e-5}]         # outside
    sp = bench.speedup_at_equal_error(rows)
    assert len(sp) == 1 and sp[0]["dt_dSDC"] == 100.0
    assert sp[0]["speedup_vs_IMEX_o2"] == pytest.approx(2 ** 0.5 / 0.5, rel=1e-3)
