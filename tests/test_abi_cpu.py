"""CPU checks of the C ABI: the library loads, exports every function that
include/lb.h declares, and validates its arguments (no GPU calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lb():
    from paper_2101_04847_amd import lb as mod
    return mod


def _declared():
    src = open(os.path.join(ROOT, "include", "lb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lb):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lb._lib, n), n
    assert sorted(lb.EXPORTS) == names


def test_header_constants_match_binding(lb):
    src = open(os.path.join(ROOT, "include", "lb.h")).read()
    consts = dict((k, int(v)) for k, v in re.findall(r"#define (LB_[A-Z0-9_]+) \(?(-?\d+)\)?", src))
    assert consts["LB_OK"] == lb.LB_OK and consts["LB_EINVAL"] == lb.LB_EINVAL
    assert consts["LB_ENOMEM"] == lb.LB_ENOMEM and consts["LB_EHIP"] == lb.LB_EHIP
    assert consts["LB_ESTATE"] == lb.LB_ESTATE and consts["LB_ENONFINITE"] == lb.LB_ENONFINITE
    assert consts["LB_EINTERNAL"] == lb.LB_EINTERNAL
    assert (consts["LB_F64"], consts["LB_F32"], consts["LB_F16S"], consts["LB_BF16S"]) == (0, 1, 2, 3)
    assert (consts["LB_FORCE_SHIFT"], consts["LB_FORCE_GUO"]) == (0, 1)
    assert (consts["LB_WALLS"], consts["LB_PERIODIC_Y"]) == (0, 1)
    assert (consts["LB_PSI_MIRROR"], consts["LB_PSI_ZERO"]) == (lb.PSI_MIRROR, lb.PSI_ZERO) == (0, 1)
    assert consts["LB_MAX_MEMBERS"] == lb.MAX_MEMBERS
    # struct sizes the binding assumes
    assert ctypes.sizeof(lb.LbMember) == 4 * 2 + 8 * 2 + 8 + 8 * 4 + 8 * 2 + 8 * 2 + 8 * 2 + 4 + 4
    assert ctypes.sizeof(lb.LbDiag) == 8 + 16 + 5 * 8 + 8
    assert ctypes.sizeof(lb.LbConfig) == 4 + 4 + 8 + 8 * 4
    assert ctypes.sizeof(lb.LbBudget) == 8 + 6 * 8
    assert ctypes.sizeof(lb.LbInterface) == 8 + 4 * 8 + 8
    assert ctypes.sizeof(lb.LbTopology) == 8 + 2 * 8
    assert ctypes.sizeof(lb.LbMixing) == 8 + 3 * 8


def _member(lb, nx=32, ny=30, **kw):
    r = np.ones((ny, nx))
    return lb.Member(nx, ny, r, r, tau=kw.pop("tau", (1.0, 1.0)), **kw)


def test_workspace_bytes_accounts_for_storage(lb):
    m = _member(lb, 100, 40)
    b64 = lb.workspace_bytes([m], storage=lb.F64)
    b32 = lb.workspace_bytes([m], storage=lb.F32)
    b16 = lb.workspace_bytes([m], storage=lb.F16S)
    pitch = 128
    pops = 2 * 9 * 40 * pitch
    assert b64 - b32 == 2 * pops * 4
    # the 16-bit modes add two FP32 site-density segments per row block
    assert b32 - b16 == 2 * pops * 2 - 2 * (2 * 40 * pitch * 4)
    assert b64 >= 2 * pops * 8 + 4 * 100 * 40 * 8


@pytest.mark.parametrize("kw,msg", [
    (dict(storage=7), "storage"),
    (dict(forcing=3), "forcing"),
    (dict(bc_y=2), "bc_y"),
    (dict(diag_trim=0), "diag_trim"),
    (dict(tile_x=100), "tile_x"),
    (dict(graph_chunk=7), "graph_chunk"),
    (dict(steps_per_pass=4), "steps_per_pass"),
    (dict(steps_per_pass=-1), "steps_per_pass"),
])
def test_config_validation(lb, kw, msg):
    c, _k = lb.make_config([_member(lb)], **kw)
    assert lb._lib.lb_workspace_bytes(ctypes.byref(c)) == 0
    assert msg in lb.last_error()


@pytest.mark.parametrize("mkw,msg", [
    (dict(tau=(0.5, 1.0)), "tau"),
    (dict(tau=(1.0, float("nan"))), "tau"),
    (dict(nx=2), "nx"),
    (dict(ny=20), "trimming"),
    (dict(G=float("inf")), "G_AB"),
    (dict(G_wall=(0.1, float("nan"))), "G_wall"),
    (dict(wall_psi=2), "wall_psi"),
])
def test_member_validation(lb, mkw, msg):
    nx = mkw.pop("nx", 32)
    ny = mkw.pop("ny", 30)
    c, _k = lb.make_config([_member(lb, nx, ny, **mkw)])
    assert lb._lib.lb_workspace_bytes(ctypes.byref(c)) == 0
    assert msg in lb.last_error()


def test_guo_needs_equal_tau(lb):
    c, _k = lb.make_config([_member(lb, tau=(1.0, 0.8))], forcing=lb.FORCE_GUO)
    assert lb._lib.lb_workspace_bytes(ctypes.byref(c)) == 0
    assert "Guo" in lb.last_error()


def test_init_rejects_null_and_small_workspace(lb):
    c, _k = lb.make_config([_member(lb)])
    h = ctypes.c_void_p()
    assert lb._lib.lb_init(ctypes.byref(c), None, 1 << 30, None, ctypes.byref(h)) == lb.LB_EINVAL
    assert "workspace" in lb.last_error()
    need = lb._lib.lb_workspace_bytes(ctypes.byref(c))
    # a fake, aligned, never dereferenced address: the size check comes first
    assert lb._lib.lb_init(ctypes.byref(c), ctypes.c_void_p(1 << 20), need - 1, None, ctypes.byref(h)) == lb.LB_ENOMEM
    assert lb._lib.lb_init(ctypes.byref(c), ctypes.c_void_p((1 << 20) + 8), need, None, ctypes.byref(h)) == lb.LB_EINVAL
    assert "aligned" in lb.last_error()
    assert lb._lib.lb_init(None, ctypes.c_void_p(1 << 20), need, None, ctypes.byref(h)) == lb.LB_EINVAL


def test_unknown_handle_is_rejected(lb):
    bogus = ctypes.c_void_p(0x1234)
    assert lb._lib.lb_step(bogus, 1) == lb.LB_ESTATE
    assert lb._lib.lb_time(bogus) == -1
    assert lb._lib.lb_steps_per_pass(bogus) == lb.LB_ESTATE
    assert lb._lib.lb_destroy(bogus) == lb.LB_ESTATE
    assert lb._lib.lb_destroy(None) == lb.LB_ESTATE
    d = lb.LbDiag()
    assert lb._lib.lb_diagnostics(bogus, 0, ctypes.byref(d), None) == lb.LB_ESTATE
    b = lb.LbBudget()
    assert lb._lib.lb_energy_budget(bogus, 0, ctypes.byref(b)) == lb.LB_ESTATE
    r = lb.LbInterface()
    assert lb._lib.lb_interface_length(bogus, 0, ctypes.byref(r)) == lb.LB_ESTATE
    tp = lb.LbTopology()
    assert lb._lib.lb_components(bogus, 0, ctypes.byref(tp)) == lb.LB_ESTATE
    assert lb._lib.lb_fields(bogus, 0, None, None, None, None) == lb.LB_ESTATE
    assert "live" in lb.last_error()


def test_oracle_is_not_imported_by_the_product(lb):
    """The product package must not reach into the test oracle."""
    pkg = os.path.join(ROOT, "paper_2101_04847_amd")
    for dirpath, _d, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "orc_" not in text, fn


@pytest.mark.parametrize("header,struct", [("lb.h", "lb_config"), ("lb3.h", "lb3_config")])
@pytest.mark.parametrize("lang", ["c", "c++"])
def test_header_compiles_cleanly(lang, header, struct, tmp_path):
    """include/lb.h and include/lb3.h are self-contained and warning-free as
    C and C++."""
    import subprocess
    src = tmp_path / ("t.c" if lang == "c" else "t.cpp")
    src.write_text(f'#include "{header}"\nint main(void) {{ return (int)sizeof({struct}); }}\n')
    cc = "gcc" if lang == "c" else "g++"
    r = subprocess.run([cc, "-Wall", "-Wextra", "-Werror", "-fsyntax-only", "-I", os.path.join(ROOT, "include"),
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


# --- the 3D (D3Q19) entry points ---------------------------------------------

@pytest.fixture(scope="module")
def lb3(lb):
    from paper_2101_04847_amd import lb3 as mod
    return mod


def test_lb3_declared_symbols_are_exported(lb3):
    src = open(os.path.join(ROOT, "include", "lb3.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = sorted(set(re.findall(r"\b(lb3_[a-z_]+)\s*\(", src)))
    assert len(names) >= 9
    assert sorted(lb3.EXPORTS3) == names
    for n in names:
        assert hasattr(lb3._lib, n), n
    assert ctypes.sizeof(lb3.Lb3Config) == 8 * 4 + 2 * 8 + 8 + 6 * 8 + 2 * 8
    assert ctypes.sizeof(lb3.Lb3Diag) == 8 + 2 * 8 + 8 + 8 + 4 + 4


@pytest.mark.parametrize("kw,msg", [
    (dict(storage=2), "storage"),
    (dict(nz=2), "nz"),
    (dict(diag_trim=5), "diag_trim"),
    (dict(tau=(0.5, 1.0)), "tau"),
    (dict(G=float("nan")), "G_AB"),
    (dict(bc_y=3), "bc_y"),
    (dict(nx=8_000_000, ny=3, nz=3), "row block"),
])
def test_lb3_config_validation(lb, lb3, kw, msg):
    nx, ny, nz = kw.pop("nx", 8), kw.pop("ny", 10), kw.pop("nz", 6)
    r = np.ones((nz, ny, nx))
    c, _k = lb3.make_config3(nx, ny, nz, r, r, **kw)
    assert lb3._lib.lb3_workspace_bytes(ctypes.byref(c)) == 0
    assert msg in lb.last_error()


def test_lb3_workspace_and_bogus_handle(lb, lb3):
    r = np.ones((6, 10, 100))
    c64, _a = lb3.make_config3(100, 10, 6, r, r, storage=lb.F64)
    c32, _b = lb3.make_config3(100, 10, 6, r, r, storage=lb.F32)
    pops = 2 * 19 * 10 * 6 * 128
    b64 = lb3._lib.lb3_workspace_bytes(ctypes.byref(c64))
    b32 = lb3._lib.lb3_workspace_bytes(ctypes.byref(c32))
    assert b64 - b32 == 2 * pops * 4
    assert b64 >= 2 * pops * 8 + 5 * 100 * 10 * 6 * 8
    bogus = ctypes.c_void_p(0x1234)
    assert lb3._lib.lb3_step(bogus, 1) == lb.LB_ESTATE
    assert lb3._lib.lb3_time(bogus) == -1
    assert lb3._lib.lb3_destroy(bogus) == lb.LB_ESTATE
    d = lb3.Lb3Diag()
    assert lb3._lib.lb3_diagnostics(bogus, ctypes.byref(d)) == lb.LB_ESTATE
    assert lb3._lib.lb3_fields(bogus, None, None, None, None, None) == lb.LB_ESTATE


# --- the C ABI from a plain C program (tests/c/lb_c_driver.c) ----------------

def _c_driver():
    import importlib.util
    spec = importlib.util.spec_from_file_location("build_driver", os.path.join(ROOT, "tests", "c", "build_driver.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _write_driver_input(path, nx, ny, tau, G, g, rA, rB):
    with open(path, "wb") as fh:
        fh.write(np.array([nx, ny], dtype=np.int32).tobytes())
        fh.write(np.array([tau[0], tau[1], G, g[0][0], g[0][1], g[1][0], g[1][1]], dtype=np.float64).tobytes())
        fh.write(np.ascontiguousarray(rA, dtype=np.float64).tobytes())
        fh.write(np.ascontiguousarray(rB, dtype=np.float64).tobytes())


def test_c_driver_compiles_warning_free(lb, tmp_path):
    """The C drivers build with gcc -Wall -Wextra -Werror against include/lb.h
    and include/lb3.h and link liblb.so and the HIP runtime."""
    d = _c_driver()
    assert os.path.exists(d.build(str(tmp_path / "drv")))
    assert os.path.exists(d.build(str(tmp_path / "drv3"), d.SRC3))


def test_c_driver_reports_invalid_configuration(lb, tmp_path):
    """From C, an invalid member (tau_A = 0.4 <= 1/2) makes lb_workspace_bytes
    return 0 with a message from lb_last_error; no device call is made."""
    import subprocess
    d = _c_driver()
    exe = d.build()
    nx, ny = 16, 12
    r = np.ones((ny, nx))
    _write_driver_input(tmp_path / "in.bin", nx, ny, (0.4, 1.0), 1.0, ((0, 0), (0, 0)), r, r)
    p = subprocess.run([exe, str(tmp_path / "in.bin"), str(tmp_path / "out.bin"), "3", "0", "0", "1"],
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 1, p.stderr
    assert "tau" in p.stderr
    rc = np.frombuffer(open(tmp_path / "out.bin", "rb").read(28), dtype=np.int32)
    assert rc[0] == lb.LB_EINVAL
    q = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert q.returncode == 2 and "usage" in q.stderr



def test_c_driver_3d_reports_invalid_configuration(lb, tmp_path):
    """From C, lb3_workspace_bytes rejects tau_B = 0.5 with a message."""
    import subprocess
    d = _c_driver()
    exe = d.build(d.EXE3, d.SRC3)
    nx, ny, nz = 8, 6, 5
    r = np.ones((nz, ny, nx))
    with open(tmp_path / "in.bin", "wb") as fh:
        fh.write(np.array([nx, ny, nz], dtype=np.int32).tobytes())
        fh.write(np.array([1.0, 0.5, 1.0, 0, 0, 0, 0, 0, 0], dtype=np.float64).tobytes())
        fh.write(r.tobytes())
        fh.write(r.tobytes())
    p = subprocess.run([exe, str(tmp_path / "in.bin"), str(tmp_path / "out.bin"), "3", "0", "0", "0"],
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 1, p.stderr
    assert "tau" in p.stderr
    rc = np.frombuffer(open(tmp_path / "out.bin", "rb").read(28), dtype=np.int32)
    assert rc[0] == lb.LB_EINVAL


def test_tile_cache_file_logic(tmp_path):
    """The persisted tile cache (host code of liblb): round trip of choices
    under several keys, a corrupt file ignored and rewritten, and the cache
    switched off by LB_TILE_CACHE=off, and truncated or corrupted files read
    without fault (a C++ check built with g++ under the address and
    undefined-behaviour sanitizers)."""
    import subprocess
    exe = tmp_path / "tune_cache_check"
    src = os.path.join(ROOT, "tests", "c", "tune_cache_check.cpp")
    inc = os.path.join(ROOT, "paper_2101_04847_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-Wall", "-Wextra", "-Werror", "-I", inc, "-o", str(exe), src], check=True)
    r = subprocess.run([str(exe), str(tmp_path / "sub" / "tiles.json")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "ok"
    text = (tmp_path / "sub" / "tiles.json").read_text()
    import json
    assert set(json.loads(text)) == {"k4"}
