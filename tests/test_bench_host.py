"""Host-side logic of bench.py (no GPU): the single-GPU refusal, the
algorithmic byte counts behind the roofline figures, and the fraction of
the HBM peak they imply."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_update():
    # 2 components x 9 populations x (read + write) x element size, plus the
    # two FP32 site densities of the 16-bit modes
    assert bench.BYTES_PER_LU == {"f64": 288, "f32": 144, "f16s": 2 * (18 * 2 + 2 * 4), "bf16s": 88}
    # 3D: 2 x 19 populations read and written once (fused), plus a second
    # read and the density buffer in the two-pass step
    assert bench.BYTES_PER_LU_3D_FUSED == {"f64": 608, "f32": 304}
    assert bench.BYTES_PER_LU_3D == {"f64": 944, "f32": 488}


def test_hbm_fraction():
    # 10000 x 5000 FP64, two steps per pass at 1.7838 ms per step: 14.4 GB per 3.5676 ms
    assert bench.hbm_frac("f64", 2, 1.7838, 5e7) == pytest.approx(14.4e9 / 3.5676e-3 / 8e12, abs=1e-4)
    assert bench.hbm_frac("f64", 1, 2.7186, 5e7) == pytest.approx(0.6621, abs=1e-4)


def test_traffic_record_missing_is_null():
    assert bench.measured_traffic("step2", "f64", 123, 45) is None


def test_traffic_record_needs_current_sources_and_tile(tmp_path, monkeypatch):
    """A counter record counts only for the kernel sources it was taken
    from and for the tile it names."""
    import json
    from paper_2101_04847_amd.profiling import kernel_source_hash
    (tmp_path / "profiles").mkdir()
    rec = {"source_hash": kernel_source_hash(), "bytes_per_launch": 123, "tile": [58, 8]}
    path = tmp_path / "profiles" / "step2_f64_64x32_traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("step2", "f64", 64, 32, tile=[58, 8]) == 123
    assert bench.measured_traffic("step2", "f64", 64, 32) == 123
    assert bench.measured_traffic("step2", "f64", 64, 32, tile=[58, 10]) is None
    other = dict(rec, tile=[58, 10], bytes_per_launch=456)
    path.write_text(json.dumps([rec, other]))
    assert bench.measured_traffic("step2", "f64", 64, 32, tile=[58, 10]) == 456
    assert bench.measured_traffic("step2", "f64", 64, 32, tile=[58, 12]) is None
    rec["source_hash"] = "0" * 16
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("step2", "f64", 64, 32, tile=[58, 8]) is None


def test_cpu_baseline_reports_all_cores_and_one_thread():
    """The oracle leg of bench.py on a small lattice: the rate on every host
    thread and on one thread, and the thread count restored afterwards."""
    import oracle
    from paper_2101_04847_amd import inputs
    before = oracle.threads()
    r = bench.cpu_baseline(inputs.Workload(96, 40, seed=3, name="tiny"), target_s=0.05)
    assert r["kind"] == "oracle" and r["unit"] == "MLUPS" and r["value"] > 0
    assert r["cores"] == before == oracle.threads()
    assert r["single_thread"]["value"] > 0 and r["single_thread"]["unit"] == "MLUPS"


def test_sq_summary_arithmetic(tmp_path):
    """The shader-sequencer summary: shares of wave cycles and the VALU busy
    fraction SQ_ACTIVE_INST_VALU x 4 / n_simd / GRBM_GUI_ACTIVE, as means over
    the dispatches of the matching kernel only."""
    from paper_2101_04847_amd import profiling
    vals = {"SQ_WAVE_CYCLES": 1000.0, "SQ_WAIT_INST_ANY": 400.0, "SQ_WAIT_ANY": 500.0, "SQ_ACTIVE_INST_ANY": 300.0,
            "SQ_ACTIVE_INST_VALU": 2560.0, "SQ_ACTIVE_INST_VMEM": 50.0, "SQ_INSTS_VALU": 7.0, "GRBM_GUI_ACTIVE": 20.0}
    lines = ["Kernel_Name,Counter_Name,Counter_Value"]
    for k, v in vals.items():
        lines.append(f'"void lbk::k_step2<0, 0, 0>(x)",{k},{v}')
        lines.append(f'"void lbk::k_step2<0, 0, 0>(x)",{k},{v * 3}')
        lines.append(f'"other",{k},1')
    path = tmp_path / "c.csv"
    path.write_text("\n".join(lines) + "\n")
    s = profiling.sq_summary(str(path), r"k_step2<0, 0, 0>", 1024, 8)
    assert s["dispatches"] == 2
    assert s["wait_dependency"] == pytest.approx(0.4) and s["issue_any"] == pytest.approx(0.3)
    assert s["cycles"] == pytest.approx(20.0 * 2 / 8)
    assert s["valu_busy"] == pytest.approx(2560.0 * 2 * 4 / 1024 / (20.0 * 2 / 8))
    assert s["valu_busy_from_insts"] == pytest.approx(7.0 * 2 * 4 / 1024 / (20.0 * 2 / 8))


def test_profile_commands_are_current():
    """Every command a profile summary gives runs committed code with options
    that exist: bench.py flags parse, profiling subcommands exist, and the
    programs named are built by build()."""
    import glob
    import os
    import re
    import shlex
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subs = {"trace", "traffic", "sq", "copy"}
    seen = 0
    for md in sorted(glob.glob(os.path.join(root, "profiles", "*.md"))):
        for line in open(md):
            if not line.startswith("    ") or line.strip().startswith("|"):
                continue
            cmd = re.sub(r"<[^>]*>", "X", line.strip().rstrip("\\").strip())
            if "python bench.py" in cmd:
                args = shlex.split(cmd.split("python bench.py", 1)[1])
                bench.parser().parse_args(args)
                seen += 1
            elif "python -m paper_2101_04847_amd.profiling" in cmd:
                assert cmd.split("python -m paper_2101_04847_amd.profiling", 1)[1].split()[0] in subs, (md, cmd)
                seen += 1
            elif cmd.startswith("./"):
                exe = cmd.split()[0][2:]
                assert exe == "paper_2101_04847_amd/bw_probe", (md, cmd)
                assert os.path.exists(os.path.join(root, "paper_2101_04847_amd", "csrc", "bw_probe.hip"))
                seen += 1
    assert seen >= 20
