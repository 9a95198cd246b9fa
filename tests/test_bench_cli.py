"""bench.py's command line (CPU): more than one GPU is refused with a message
before any GPU work, and the workloads it names are the ones it can run."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_help_lists_the_workloads():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 0
    for name in ("hard_cube", "batch64", "film", "polycrystal", "--jmax", "--poisson-prec"):
        assert name in r.stdout, name


def test_curve_in_pieces_resumes_where_it_stopped(tmp_path, monkeypatch):
    """A curve timed in pieces: the first run stops at its time limit after one
    piece and saves the state; the second resumes at the next field with the
    saved m and finishes, counting every field once."""
    import json
    import types

    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    import bench

    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)

    class FakeCtx:
        def __init__(self):
            self.pieces = []

        def reset_warm_start(self):
            pass

        def curve(self, m, f, opts=None):
            self.pieces.append(len(f))
            m += 1.0
            st = dict(evals=2, nli=1, li=3, mi=10, restarts=0, fallbacks=0, status=0)
            return dict(stats=[st] * len(f), E=np.zeros(len(f)), m_avg=np.ones((len(f), 3)))

    args = types.SimpleNamespace(state=str(tmp_path / "state.npz"), time_limit=1e-12, progress_every=3,
                                 workload="polycrystal", precision="fp32", poisson_prec="amg")
    fields = [[0.0, 0.0, -0.01 * k] for k in range(10)]
    m0 = torch.zeros(4, 3, dtype=torch.float64)
    m = torch.empty_like(m0)
    info = dict(n_mag=4, n_pot=9, nnz_K=20)
    w = types.SimpleNamespace(fields=fields)
    first = FakeCtx()
    bench.curve_in_pieces(args, first, w, fields, None, m, m0, info, 4, (16, [1]))
    assert first.pieces == [3]
    st = np.load(args.state)
    assert int(st["next_field"]) == 3 and int(st["runs"]) == 1
    np.testing.assert_array_equal(st["m"], np.ones((4, 3)))
    args.time_limit = 0.0
    second = FakeCtx()
    m.zero_()
    capsys_out = []
    monkeypatch.setattr("builtins.print", lambda *a, **k: capsys_out.append(a[0]))
    bench.curve_in_pieces(args, second, w, fields, None, m, m0, info, 4, (16, [1]))
    assert second.pieces == [3, 3, 1]
    np.testing.assert_array_equal(m.numpy(), np.full((4, 3), 4.0))
    out = json.loads(capsys_out[-1])
    assert out["counters"]["nli"] == 10 and out["counters"]["mi"] == 100
    assert "2 runs" in out["config"]["workload"]


def test_counter_traffic_is_reported_only_for_the_profiled_kernel_source(tmp_path, monkeypatch):
    """roofline.traffic comes from a committed counter summary only while the
    kernel source still hashes to the one profiled; a changed source, another
    precision or a missing summary gives null."""
    import hashlib

    sys.path.insert(0, ROOT)
    import bench

    src = tmp_path / "kernel.hip"
    src.write_text("// a kernel\n")
    h = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    summ = tmp_path / "traffic.txt"
    summ.write_text(f"# counters\nsource_sha256_prefix {h}\nprecision fp32\ntraffic_bytes_per_iteration 1234.5\n")
    monkeypatch.setitem(bench.TRAFFIC, ("film", "jacobi"), (str(summ), str(src)))
    assert bench.measured_traffic("film", "fp32", "jacobi") == 1234.5
    assert bench.measured_traffic("film", "fp64", "jacobi") is None
    src.write_text("// a kernel, changed\n")
    assert bench.measured_traffic("film", "fp32", "jacobi") is None
    monkeypatch.setitem(bench.TRAFFIC, ("film", "jacobi"), (str(tmp_path / "missing.txt"), str(src)))
    assert bench.measured_traffic("film", "fp32", "jacobi") is None
    assert bench.measured_traffic("batch64", "fp32", "jacobi") is None


def test_committed_traffic_summaries_are_well_formed():
    """Every committed counter summary names the sha256 prefix of the kernel
    source it was taken on and a positive byte count; the bench line reports
    its traffic only while the prefix matches the current source (null once
    the kernel has changed since the counters were taken)."""
    import hashlib

    sys.path.insert(0, ROOT)
    import bench

    for key, (path, src) in bench.TRAFFIC.items():
        kv = dict(line.split(None, 1) for line in open(path) if line.strip() and not line.startswith("#"))
        assert len(kv["source_sha256_prefix"].strip()) == 16 and float(kv["traffic_bytes_per_iteration"]) > 0, key
        assert kv["precision"].strip() in ("fp32", "fp64"), key
