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
