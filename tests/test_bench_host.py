"""Host logic of bench.py that runs without a GPU: the HBM-traffic lookup
from a committed counter summary (used only while the kernel source is the
one the counters were taken on) and the refusal of more than one GPU."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write(path, text):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write(text)


def test_traffic_lookup_follows_the_source_hash(tmp_path, monkeypatch):
    src = "kern.hip"
    _write(str(tmp_path / src), "kernel source v1\n")
    sha = hashlib.sha256(b"kernel source v1\n").hexdigest()
    _write(str(tmp_path / "profiles" / "p.md"),
           f"# counters\n\n```\nkernel: k\ntraffic_bytes_per_launch: 1234567\nsource_sha256: {sha}\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("p.md", src) == 1234567.0
    _write(str(tmp_path / src), "kernel source v2\n")          # the kernel changed: no figure
    assert bench.measured_traffic("p.md", src) is None
    assert bench.measured_traffic("missing.md", src) is None


def test_committed_summary_is_readable():
    """The committed adjoint summary parses; its figure is returned exactly
    when its hash matches the current source."""
    text = open(os.path.join(ROOT, "profiles", "k_sf_adjoint_single_grain_hbm_counters.md")).read()
    vals = dict(l.split(": ", 1) for l in text.splitlines() if l.startswith(("traffic_bytes_per_launch", "source_sha256")))
    assert float(vals["traffic_bytes_per_launch"]) > 0 and len(vals["source_sha256"]) == 64
    src = os.path.join("paper_2009_00735_amd", "csrc", "refine.hip")
    sha = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
    got = bench.measured_traffic("k_sf_adjoint_single_grain_hbm_counters.md", src)
    assert got == (float(vals["traffic_bytes_per_launch"]) if sha == vals["source_sha256"] else None)


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_structure_factor_accounting():
    """Arithmetic per term: phase 1, C and S 2, the shared dot product
    5 / n_freq, the adjoint's P and Q 12; sine and cosine are not flops.
    Antipodal pairs of the icosphere share one evaluation."""
    import bench
    from paper_2009_00735_amd import synth
    assert bench.sf_flop_per_term(4, True) == 16.25
    assert bench.sf_flop_per_term(4, False) == 4.25
    assert bench.evaluated_directions(synth.icosphere(3)) == 321
    assert bench.evaluated_directions(synth.icosphere(5)) == 5121
