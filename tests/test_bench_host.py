"""Host logic of bench.py (no GPU): the single-GPU contract, the roofline
record and the HBM traffic record lookup."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_multi_gpu_request_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_sap_flops_per_site():
    # 4^4 blocks: 3/4 of the hops stay inside the block
    assert bench.sap_flops_per_site((4, 4, 4, 4), 4) == 1848 + 4 * (504 + 0.75 * 1320 + 336) + 24
    # single-site blocks: the MR steps see the clover term only
    assert bench.sap_flops_per_site((1, 1, 1, 1), 4) == 1848 + 4 * (504 + 336) + 24
    # more MR steps, more work
    assert bench.sap_flops_per_site((4, 4, 4, 4), 5) > bench.sap_flops_per_site((4, 4, 4, 4), 4)


def test_dominant_roofline_takes_the_longest_priced_class():
    w = bench.WORKLOADS["c3"]
    V = 32 ** 3 * 64
    kt = {"sap": (300.0, 60, 1200), "dslash": (20.0, 12, 144), "outer_gs": (900.0, 12, 144),
          "restrict": (0.0, 0, 0)}
    r = bench.dominant_roofline(w, kt, 2)
    assert r["kernel"] == "sap" and r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    work = 1200 * (V / 2) * bench.sap_flops_per_site(w["block"], 4)
    assert r["achieved"] == pytest.approx(work / 0.3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["avg_launch_ms"] == pytest.approx(5.0) and r["launches"] == 60
    assert r["algorithmic_per_launch"] == pytest.approx(work / 60)
    assert r["frac_unpacked"] == pytest.approx(r["achieved"] / bench.FP32_UNPACKED_TFLOPS)
    # a memory-bound class when it takes longer
    r = bench.dominant_roofline(w, {"sap": (1.0, 1, 1), "dslash": (20.0, 12, 144)}, 2)
    assert r["kernel"] == "dslash" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx((12 * V * 1152 + 144 * V * (12 * 8 + 192)) / 0.02 / 1e9)


def test_traffic_record_applies_only_to_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    srcs = ["k_sap.hip", "dirac_device.h"]
    good = {"class": "sap", "workload": "wl", "kernel": "k", "bytes_per_launch": 123, "sources": srcs,
            "sources_sha256": bench.sources_digest(srcs)}
    stale = dict(good, workload="wl2", sources_sha256="0" * 64)
    f = tmp_path / "rec.txt"
    f.write_text("header\nrecord: %s\nrecord: %s\n" % (json.dumps(good), json.dumps(stale)))
    monkeypatch.setattr(bench, "TRAFFIC_RECORDS", str(f))
    assert bench.measured_traffic("sap", "wl") == 123
    assert bench.measured_traffic("sap", "wl2") is None  # sources changed since
    assert bench.measured_traffic("dslash", "wl") is None
    monkeypatch.setattr(bench, "TRAFFIC_RECORDS", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("sap", "wl") is None


def test_committed_traffic_record_is_well_formed():
    with open(bench.TRAFFIC_RECORDS) as fh:
        recs = [json.loads(l[len("record: "):]) for l in fh.read().splitlines() if l.startswith("record: ")]
    assert recs
    for r in recs:
        assert {"class", "workload", "kernel", "bytes_per_launch", "sources", "sources_sha256"} <= set(r)
        assert r["bytes_per_launch"] > 0 and len(r["sources_sha256"]) == 64
        assert r["workload"] in {w["name"] for w in bench.WORKLOADS.values()}


def test_low_mode_helpers():
    """The host linear algebra of the low-mode comparison: Cholesky QR rows
    are orthonormal and span the input; gamma5 flips spins 0 and 1 only; the
    Rayleigh-Ritz vectors built the way low_modes builds them have |A v_k|^2
    equal to the Ritz values (here with a dense A)."""
    import torch
    torch.manual_seed(0)
    n, shape = 4, (4, 2, 2, 2, 2, 4, 3)
    V = torch.randn(shape, dtype=torch.complex128) * torch.arange(1, n + 1, dtype=torch.float64).reshape(n, 1, 1, 1,
                                                                                                       1, 1, 1)
    Q = bench._orthonormal_rows(torch, V)
    M = Q.reshape(n, -1)
    assert (M @ M.conj().T - torch.eye(n)).abs().max() < 1e-12
    P = V.reshape(n, -1)
    assert ((P @ M.conj().T) @ M - P).abs().max() < 1e-12 * P.abs().max()
    g = bench._gamma5(torch, V)
    assert torch.equal(g[..., :2, :], -V[..., :2, :]) and torch.equal(g[..., 2:, :], V[..., 2:, :])
    A = torch.randn(M.shape[1], M.shape[1], dtype=torch.complex128)
    W = (A @ M.T).T
    ev, Qh = torch.linalg.eigh(torch.matmul(W.conj(), W.transpose(0, 1)))
    R = torch.matmul(Qh.transpose(0, 1), M)
    WR = (A @ R.T).T
    for k in range(n):
        assert abs(WR[k].norm() ** 2 - ev[k]) < 1e-9 * ev[-1]
