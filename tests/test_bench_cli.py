"""bench.py on the CPU: the multi-GPU refusal, the oracle baseline leg on a
small grid, and the comment-insensitive source hash that ties committed
counter summaries to the kernels they were taken on."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1905_05727_amd import scenario as S  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_cpu_baseline_leg_on_a_small_grid():
    sc = S.single_bubble(nx=96, ny=48, radius=8.0, centre=(50.0, 24.0), shock_x=30.0)
    out = bench.cpu_baseline(sc, 3)
    assert out["kind"] == "oracle" and out["unit"] == "cell-updates/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "96x48" in out["sample"]
    one = bench.cpu_one_core(sc, 24, 1)
    assert one["cores"] == 1 and one["value"] > 0 and "96x24" in one["sample"]
    import oracle
    assert oracle.num_threads() >= 1      # back to all processors afterwards


def test_oracle_thread_count_changes_no_result():
    import oracle
    sc = S.single_bubble(nx=80, ny=40, radius=8.0, centre=(44.0, 20.0), shock_x=24.0)
    res = []
    for n in (1, 0):
        oracle.set_threads(n)
        o = bench.oracle_of(sc)
        o.run(5)
        res.append(o.U.copy())
    assert np.array_equal(res[0], res[1])


def test_cpu_baseline_leg_for_each_liquid():
    # the regular-array section times the oracle per liquid with the
    # scenario's own materials and boundaries; a cropped copy keeps it short
    for name, kw in bench.LIQUIDS:
        sc = S.regular_array(length=700, strip=100, **kw)
        out = bench.cpu_baseline(sc, 1)
        d = bench.oracle_diagnostics(sc, 64)
        assert set(d["ms"]) == {"y_averages", "integrals", "pdf_p", "pdf_rho"}
        assert out["value"] > 0, name
        assert sc.prim.shape[0] == (7 if kw.get("reactive") else 6)


def test_source_hash_ignores_comments_and_whitespace(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1905_05727_amd", "csrc")
    h0 = bench.kernel_source_hash()
    fake = tmp_path / "paper_1905_05727_amd"
    (fake / "csrc").mkdir(parents=True)
    for f in os.listdir(src):
        if f.endswith((".h", ".hip")):
            text = open(os.path.join(src, f)).read()
            if f == "meso_device.h":
                text = "// a new comment\n/* and a block\n comment */\n" + text.replace(";", " ;")
            (fake / "csrc" / f).write_text(text)
    (fake / "build.py").write_bytes(open(os.path.join(ROOT, "paper_1905_05727_amd",
                                                      "build.py"), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h0
    (fake / "csrc" / "meso_device.h").write_text(
        (fake / "csrc" / "meso_device.h").read_text().replace("kHalo", "kHalo2"))
    assert bench.kernel_source_hash() != h0


def test_bytes_per_cell_and_peaks():
    # one read and one write of the 6-plane state per step: 2 x 6 x 8 B, 2 x 6 x 4 B in FP32
    assert bench.BYTES_PER_CELL == {"fp64": 96, "fp64_fast": 96, "fp32_fp64acc": 96,
                                    "fp32": 48}
    assert abs(bench.VALU_ISSUE_PEAK - 39.3216) < 1e-9
    assert np.isclose(bench.HBM_PEAK_GBS, 8000.0)


def test_headline_is_an_fp64_mode():
    ap_defaults = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                                 capture_output=True, text=True, timeout=120).stdout
    assert "--headline" in ap_defaults
    assert bench.DTYPE["fp64_fast"] == "f64" and bench.DTYPE["fp64"] == "f64"
