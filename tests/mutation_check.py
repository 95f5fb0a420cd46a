"""Mutation check of the oracle's pins (CPU only; not collected by pytest).

Each entry plants one plausible mistake in a temporary copy of ``oracle/``
(never in the repository's own files) and runs the oracle's CPU tests on
that copy; a mistake that no test catches is reported.  Left out: the
stored golden series (written by the oracle itself, so it would catch any
change of the dynamics without saying which pin holds) and, for the 2D
oracle, the projection of the 3D oracle onto it.

    python tests/mutation_check.py               # every entry, 4 workers
    python tests/mutation_check.py -j 2 bgk_sign ek_half

Exit status 1 if any mistake passes.  A full run takes about 20 minutes with
4 workers on 8 cores (most entries are caught within seconds; the slowest run the
whole oracle suite).
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (oracle file, name, text, replacement): each text occurs once in its file
MUTATIONS = [
    ('orc.c', 'feq_4.5', '4.5 * cv * cv', '4.0 * cv * cv'),
    ('orc.c', 'feq_vv', '- 1.5 * vv', '- 1.0 * vv'),
    ('orc.c', 'sc_sign_x', '(-p->G * sx + p->g[2 * s + 0])', '(p->G * sx + p->g[2 * s + 0])'),
    ('orc.c', 'sc_sign_y', '(-p->G * sy + p->g[2 * s + 1])', '(p->G * sy + p->g[2 * s + 1])'),
    ('orc.c', 'sc_own_component', 'rho + (size_t)(1 - s) * n;', 'rho + (size_t)s * n;'),
    ('orc.c', 'sc_no_weight', 'sx += W[i] * ps * CX[i];', 'sx += ps * CX[i];'),
    ('orc.c', 'shift_no_tau', 'vx = ux + tau * ax[s * n + k];', 'vx = ux + ax[s * n + k];'),
    ('orc.c', 'shift_no_tau_y', 'vy = uy + tau * ay[s * n + k];', 'vy = uy + ay[s * n + k];'),
    ('orc.c', 'vel_no_itau', 'double den = rA * itau[0] + rB * itau[1];', 'double den = rA + rB;'),
    ('orc.c', 'bounce_no_opp', 'fout[fidx(p, s, OPP[i], y, x)] = post;', 'fout[fidx(p, s, i, y, x)] = post;'),
    ('orc.c', 'guo_coef', '(1.0 - 0.5 / tau)', '(1.0 - 0.5 * tau)'),
    ('orc.c', 'guo_9', 'double ex = 3.0 * (CX[i] - ux) + 9.0 * cu * CX[i];', 'double ex = 3.0 * (CX[i] - ux) + 3.0 * cu * CX[i];'),
    ('orc.c', 'guo_u_half', 'ux = (jx[k] + jx[n + k] + 0.5 * (FxA + FxB)) / rt;\n                uy', 'ux = (jx[k] + jx[n + k] + (FxA + FxB)) / rt;\n                uy'),
    ('orc.c', 'bgk_sign', 'double post = fi - omega * (fi - feq[i]);', 'double post = fi - omega * (feq[i] - fi);'),
    ('orc.c', 'stream_dir_y', 'int yd = y + CY[i];', 'int yd = y - CY[i];'),
    ('orc.c', 'psi_mirror_row', 'y = y < 0 ? 0 : p->ny - 1;', 'y = y < 0 ? 1 : p->ny - 2;'),
    ('orc.c', 'wall_force_sign', '- p->Gw[s] * wy;', '+ p->Gw[s] * wy;'),
    ('orc.c', 'ek_half', 'nsum_add(&ek, 0.5 * rt *', 'nsum_add(&ek, rt *'),
    ('orc.c', 'ep_sign', 'nsum_add(&ep, -yj * fy_ext);', 'nsum_add(&ep, yj * fy_ext);'),
    ('orc.c', 'buoy_sign', 'nsum_add(&bu, -(ux[k] * fx_ext + uy[k] * fy_ext));', 'nsum_add(&bu, (ux[k] * fx_ext + uy[k] * fy_ext));'),
    ('orc.c', 'vort_sign', 'double om = dvy_dx - dux_dy;', 'double om = dvy_dx + dux_dy;'),
    ('orc.c', 'yc_offset', 'const double yc = 0.5 * (ny - 1);', 'const double yc = 0.5 * ny;'),
    ('orc.c', 'macro_u_half', 'if (ux) ux[k] = (jx[k] + jx[n + k] + 0.5 * (FxA + FxB)) / rt;', 'if (ux) ux[k] = (jx[k] + jx[n + k] + (FxA + FxB)) / rt;'),
    ('orc.c', 'macro_uy_half', 'if (uy) uy[k] = (jy[k] + jy[n + k] + 0.5 * (FyA + FyB)) / rt;', 'if (uy) uy[k] = (jy[k] + jy[n + k] + (FyA + FyB)) / rt;'),
    ('orc.c', 'macro_force_other', 'const double FxA = rho[k] * ax[k], FxB = rho[n + k] * ax[n + k];\n        const double FyA', 'const double FxA = rho[k] * ax[k], FxB = rho[n + k] * ax[k];\n        const double FyA'),
    ('orc.c', 'trim_count', 'const double nd = (double)nx * (double)(ny - 2 * trim);', 'const double nd = (double)nx * (double)(ny - 2 * trim + 1);'),
    ('orc.c', 'umax_x_only', 'double um = sqrt(ux[k] * ux[k] + uy[k] * uy[k]);', 'double um = fabs(ux[k]);'),
    ('orc.c', 'profile_sum', 'nsum_add(&prof, rA[k] - rB[k]);', 'nsum_add(&prof, rA[k] + rB[k]);'),
    ('orc.c', 'moment_sign', 'mx += v * CX[i];', 'mx -= v * CX[i];'),
    ('orc3.c', '3d_cz_swap', 'static const int CZ[NQ3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};', 'static const int CZ[NQ3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};'),
    ('orc3.c', '3d_feq', '4.5 * cv * cv', '4.0 * cv * cv'),
    ('orc3.c', '3d_mz_sign', 'mz += v * CZ[i];', 'mz -= v * CZ[i];'),
    ('orc3.c', '3d_sz_sign', '-p->G * sz + p->g[3 * s + 2]', 'p->G * sz + p->g[3 * s + 2]'),
    ('orc3.c', '3d_uz_itau', 'const double uz = (jz[k] * itau[0] + jz[n + k] * itau[1]) / den;', 'const double uz = (jz[k] + jz[n + k]) / den;'),
    ('orc3.c', '3d_stream_z', 'zd = wrap(z + CZ[i], nz)', 'zd = wrap(z - CZ[i], nz)'),
    ('orc3.c', '3d_macro_uz', 'if (uz) uz[k] = (jz[k] + jz[n + k] + 0.5 * fz) / rt;', 'if (uz) uz[k] = (jz[k] + jz[n + k] + fz) / rt;'),
    ('budget.py', 'b_pb', 'G * CS2 / 4.0 * (rho * rho - phi * phi)', 'G * CS2 / 2.0 * (rho * rho - phi * phi)'),
    ('budget.py', 'b_kappa', 'kappa = CS2 * CS2 * G / 4.0', 'kappa = CS2 * CS2 * G / 2.0'),
    ('budget.py', 'b_iso_sign', '- 0.5 * kappa * (gx * gx + gy * gy)', '+ 0.5 * kappa * (gx * gx + gy * gy)'),
    ('budget.py', 'b_pxy_sign', 'pxy = kappa * gx * gy', 'pxy = -kappa * gx * gy'),
    ('budget.py', 'b_ktau_power', '((tau - 0.5) * (tau - 0.5))', '(tau - 0.5)'),
    ('budget.py', 'b_h_sign', 'hx = _dx(rhoA) / rhoA - _dx(rhoB) / rhoB', 'hx = _dx(rhoA) / rhoA + _dx(rhoB) / rhoB'),
    ('budget.py', 'b_sxy_sign', 'sxy = _dx(uy) + _dy(ux)', 'sxy = _dx(uy) - _dy(ux)'),
    ('budget.py', 'b_eta', 'eta = rho_mean * CS2 * (tau - 0.5)', 'eta = rho_mean * CS2 * tau'),
    ('budget.py', 'b_sxx', 'sxx = 2.0 * _dx(ux)', 'sxx = _dx(ux)'),
    ('mixing.py', 'x_six', 'h += 6.0 * c * (1.0 - c)', 'h += 4.0 * c * (1.0 - c)'),
    ('mixing.py', 'x_bulk_rows', 'return p[trim], p[ny - trim - 1]', 'return p[trim - 1], p[ny - trim]'),
    ('mixing.py', 'x_conc', 'c = (phibar - phi_lo) / (phi_hi - phi_lo)', 'c = (phibar - phi_lo) / (phi_hi + phi_lo)'),
    ('interface.py', 'i_pos_ge', 'pos = np.asarray(phi, dtype=np.float64) > 0.0', 'pos = np.asarray(phi, dtype=np.float64) >= 0.0'),
    ('interface.py', 'i_diag_swap', 'n135 = int(np.count_nonzero(right[:-1] != d[1:]))', 'n135 = int(np.count_nonzero(right[1:] != d[:-1]))'),
    ('interface.py', 'i_pi_over_4', 'return float(np.pi / 8.0 * (c["n0"]', 'return float(np.pi / 4.0 * (c["n0"]'),
    ('interface.py', 'i_no_sqrt2', '(c["n45"] + c["n135"]) / np.sqrt(2.0)', '(c["n45"] + c["n135"])'),
    ('interface.py', 'i_trim_off', 'd = pos[trim:pos.shape[0] - trim]', 'd = pos[trim - 1:pos.shape[0] - trim]'),
    ('topology.py', 't_pos_ge', 'd = phi[trim:phi.shape[0] - trim] > 0.0', 'd = phi[trim:phi.shape[0] - trim] >= 0.0'),
    ('orc.c', 'w_psi_zero', 'if (p->psi_wall) return 0.0;', 'if (0) return 0.0;'),
    ('orc.c', 'w_solid_periodic', 'return !p->periodic_y && (y < 0 || y >= p->ny);', 'return (y < 0 || y >= p->ny);'),
    ('orc.c', 'g_component_swap', 'ay[s * n + sidx(p, y, x)] = (-p->G * sy + p->g[2 * s + 1])', 'ay[s * n + sidx(p, y, x)] = (-p->G * sy + p->g[2 * (1 - s) + 1])'),
    ('orc.c', 'omega_swap', 'const double omega = itau[s];', 'const double omega = itau[1 - s];'),
    ('orc.c', 'ext_force_x', 'double fx_ext = rA[k] * p->g[0] + rB[k] * p->g[2];', 'double fx_ext = rA[k] * p->g[0] + rB[k] * p->g[0];'),
    ('orc3.c', '3d_w_edge', '1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};', '1.0 / 36.0, 1.0 / 36.0, 1.0 / 37.0};'),
]

EXTRA_TESTS = ("test_inputs.py", "test_studies_host.py")


def run_one(entry) -> tuple:
    fname, name, old, new = entry
    d = tempfile.mkdtemp(prefix="orcmut_")
    try:
        for x in ("oracle", "tests", "paper_2101_04847_amd"):
            shutil.copytree(os.path.join(ROOT, x), os.path.join(d, x),
                            ignore=shutil.ignore_patterns("__pycache__", "*.so", "bw_probe"))
        shutil.copy(os.path.join(ROOT, "pytest.ini"), d)
        path = os.path.join(d, "oracle", fname)
        with open(path) as fh:
            src = fh.read()
        if src.count(old) != 1:
            return name, None, f"text occurs {src.count(old)} times in {fname}"
        with open(path, "w") as fh:
            fh.write(src.replace(old, new))
        excl = {"test_golden_series.py"} | ({"test_oracle_3d.py"} if fname == "orc.c" else set())
        files = sorted(f for f in os.listdir(os.path.join(d, "tests"))
                       if (f.startswith("test_oracle") or f in EXTRA_TESTS) and f not in excl)
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"]
                           + ["tests/" + f for f in files], cwd=d, capture_output=True, text=True,
                           env=dict(os.environ, OMP_NUM_THREADS="2"))
        failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
        return name, r.returncode != 0, failed[0] if failed else "no test failed"
    finally:
        shutil.rmtree(d, ignore_errors=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", help="entries to run (default: all)")
    ap.add_argument("-j", "--jobs", type=int, default=4)
    args = ap.parse_args()
    todo = [m for m in MUTATIONS if not args.names or m[1] in args.names]
    missed = 0
    with ThreadPoolExecutor(max_workers=max(1, args.jobs)) as ex:
        for name, caught, info in ex.map(run_one, todo):
            print(f"{name:20s} {'caught' if caught else 'MISSED' if caught is not None else 'ERROR'}  {info}", flush=True)
            missed += not caught
    print(f"{len(todo) - missed} of {len(todo)} caught")
    return 1 if missed else 0


if __name__ == "__main__":
    sys.exit(main())
