"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message (the library has no multi-GPU path), also when a
launcher sets WORLD_SIZE."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, cwd=ROOT, env=e,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_launcher_world_size_is_refused():
    r = _run(["--gpus", "1"], env={"WORLD_SIZE": "4"})
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def _counter_csv(path, counter, rows):
    with open(path, "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (name, kib) in enumerate(rows):
            fh.write(f'{i},"{name}",{counter},{kib}\n')


def test_traffic_record_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    """summarize_counters: per-launch HBM bytes are the near kernel's average
    FETCH_SIZE and WRITE_SIZE (KiB) divided by what the same counters read for
    the 512 MiB copy over its known size; the record is used only while the
    kernel sources hash to what it holds."""
    sys.path.insert(0, ROOT)
    import bench
    near = "void bem::(anonymous namespace)::k_near<double, false, false, 4>(bem::NearLaunch)"
    copy = "void at::native::elementwise_kernel<128, 4, copy_kernel>(int)"
    f, w, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "rec.json"
    _counter_csv(f, "FETCH_SIZE", [(near, 100000), (near, 120000), (copy, 262144)])
    _counter_csv(w, "WRITE_SIZE", [(near, 1000), (near, 1000), (copy, 524288)])
    bench.summarize_counters(str(f), str(w), str(out), prec="fp64")
    import json
    rec = json.load(open(out))
    assert rec["launches"] == 2
    assert abs(rec["calibration"]["fetch_scale"] - 0.5) < 1e-15
    assert abs(rec["calibration"]["write_scale"] - 1.0) < 1e-15
    expect = 110000 * 1024 / 0.5 + 1000 * 1024 / 1.0
    assert abs(rec["hbm_bytes_per_launch"] - expect) < 1e-6 * expect
    monkeypatch.setitem(bench.TRAFFIC_FILES, "fp64", str(out))
    assert bench.measured_traffic("fp64") == rec["hbm_bytes_per_launch"]
    assert bench.measured_traffic("fp64", workload="c3") is None
    rec["source_sha256"] = "0" * 64
    json.dump(rec, open(out, "w"))
    assert bench.measured_traffic("fp64") is None


def test_valu_share_from_counters(tmp_path):
    """summarize_valu: clock = GRBM_GUI_ACTIVE / 8 XCDs / duration and VALU
    share = 4 SQ_INSTS_VALU / (1024 SIMDs x clock x duration), from a dispatch
    of 1 ms at 2 GHz whose counted instructions fill half the SIMD cycles."""
    sys.path.insert(0, ROOT)
    import bench
    dur_ns, clk = 1_000_000, 2.0e9
    gui = clk * 8 * dur_ns * 1e-9
    insts = 0.5 * 1024 * clk * dur_ns * 1e-9 / 4
    name = "void bem::(anonymous namespace)::k_near<double, false, false, 4>(bem::NearLaunch)"
    p = tmp_path / "pmc.csv"
    with open(p, "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Grid_Size,Counter_Name,Counter_Value,Start_Timestamp,End_Timestamp\n")
        for c, v in (("SQ_INSTS_VALU", insts), ("SQ_ACTIVE_INST_VALU", 1.0), ("SQ_WAVES", 20480),
                     ("GRBM_GUI_ACTIVE", gui)):
            fh.write(f'7,"{name}",1310720,{c},{v},1000,{1000 + dur_ns}\n')
    out = tmp_path / "valu.md"
    bench.summarize_valu(str(p), str(out))
    row = [l for l in open(out) if l.startswith("| `void k_near<double")][0]
    cells = [c.strip() for c in row.strip().strip("|").split("|")]
    assert cells[3] == "1000.0"      # average duration in microseconds
    assert cells[7] == "2.00"        # clock in GHz
    assert cells[8] == "0.50"        # VALU share


def test_translate_traffic_groups_by_launch_shape_and_grid(tmp_path):
    """summarize_translate: one group per (kernel, grid), average bytes per
    launch over its dispatches, scaled by the calibration copy's reading."""
    sys.path.insert(0, ROOT)
    import bench
    import json
    k128 = "void bem::(anonymous namespace)::k_translate<double, HIP_vector_type<double, 2u>, false, 128, 2>(long)"
    k256 = "void bem::(anonymous namespace)::k_translate<double, HIP_vector_type<double, 2u>, false, 256, 0>(long)"
    copy = "void at::native::elementwise_kernel<128, 4, copy_kernel>(int)"
    f, w, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "tr.json"
    for path, counter, rows in ((f, "FETCH_SIZE", [(k128, 800, 4000), (k128, 800, 6000), (k256, 900, 2000),
                                                   (k128, 100, 10), (copy, 1, 262144)]),
                                (w, "WRITE_SIZE", [(k128, 800, 10), (k128, 800, 10), (k256, 900, 20),
                                                   (k128, 100, 1), (copy, 1, 524288)])):
        with open(path, "w") as fh:
            fh.write("Dispatch_Id,Kernel_Name,Grid_Size,Counter_Name,Counter_Value\n")
            for i, (name, grid, kib) in enumerate(rows):
                fh.write(f'{i},"{name}",{grid},{counter},{kib}\n')
    bench.summarize_translate(str(f), str(w), str(out), prec="fp64")
    rec = json.load(open(out))
    got = {(g["kernel"].split("false, ")[1], g["grid"]): (g["launches"], g["fetch_bytes_per_launch"],
                                                          g["write_bytes_per_launch"]) for g in rec["groups"]}
    assert got[("128, 2>", "800")] == (2, 5000 * 1024 / 0.5, 10 * 1024.0)
    assert got[("256, 0>", "900")] == (1, 2000 * 1024 / 0.5, 20 * 1024.0)
    assert got[("128, 2>", "100")] == (1, 10 * 1024 / 0.5, 1 * 1024.0)
    assert [g["fetch_bytes_per_launch"] for g in rec["groups"]] == sorted(
        (g["fetch_bytes_per_launch"] for g in rec["groups"]), reverse=True)
