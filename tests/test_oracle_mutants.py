"""Planted mistakes in a copy of the oracle's C source, each caught by the oracle's pins.

Each case copies oracle/dwfmm_oracle.c into a temporary folder, replaces one fragment with a
plausible mistake (a dropped term, a wrong sign, index, constant or operand order), compiles the
copy with the oracle's own flags and runs the CPU pin tests named for it in a child process that
loads the copy (DWFMM_ORACLE_LIB); the case passes when those pins fail.  An unmodified copy run the
same way against every pin file passes them, so each failure comes from its planted mistake.  The
children run four at a time; everything stays on the CPU.
"""
import os
import pathlib
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor


ROOT = pathlib.Path(__file__).resolve().parents[1]
SRC = ROOT / "oracle" / "dwfmm_oracle.c"
PINS, KER, ADM = "test_oracle_pins.py", "test_oracle_kernels.py", "test_oracle_admissibility.py"
AFP, EVAL, LEB = "test_oracle_afp.py", "test_oracle_eval.py", "test_oracle_lebesgue.py"
ALL = [PINS, KER, ADM, AFP, EVAL, LEB]

# name: (fragment, replacement, occurrence of the fragment to replace, its count in the source, pins)
MUTANTS = {
    # kernels (Sec 6.2 exponential; the workloads' Matern-3/2 and Gaussian)
    "matern_sign": ("return (1.0 + s) * exp(-s);", "return (1.0 - s) * exp(-s);", 0, 1, [KER]),
    "matern_no_sqrt3": ("double s = sqrt(3.0) * sqrt(r2) / ell;", "double s = sqrt(r2) / ell;", 0, 1, [KER]),
    "gauss_ell_squared": ("return exp(-r2 / ell);", "return exp(-r2 / (ell * ell));", 0, 1, [KER]),
    "exp_of_r2": ("return exp(-sqrt(r2) / ell);", "return exp(-r2 / ell);", 0, 1, [KER]),
    "distance_index": ("double t = x[k] - y[k];", "double t = x[k] - y[0];", 0, 1, [KER]),
    # dimension weights (Thm 4.6, Sec 6.2, readings R1/R2)
    "r1_natural_log": ("double w = log2(bmax / b[k]);", "double w = log(bmax / b[k]);", 0, 1, [PINS]),
    "r2_dropped_one": ("omega[k] = 1.0 + log2(bmax / b[k]);", "omega[k] = log2(bmax / b[k]);", 0, 1, [PINS]),
    "r3_dropped_e": ("omega[k] = log(exp(1.0) * g_rho(tk) / g_rho(t1));",
                     "omega[k] = log(g_rho(tk) / g_rho(t1));", 0, 1, [PINS]),
    "rho_coefficient": ("sqrt(1.0 + 4.0 * tau * tau)", "sqrt(1.0 + 2.0 * tau * tau)", 0, 1, [PINS]),
    # index set (Sec 4): the boundary sum omega.alpha = q belongs to the set
    "index_set_strict": ("if (used > rem + 1e-9) break;", "if (used >= rem - 1e-9) break;", 0, 1, [PINS]),
    # nodes and basis (Sec 5.2)
    "chebyshev_extrema": ("t[j] = (1.0 - cos((2.0 * j + 1.0) * pi / (2.0 * n))) / 2.0;",
                          "t[j] = (1.0 - cos(j * pi / (n - 1.0))) / 2.0;", 0, 1, [PINS]),
    "leja_start_at_edge": ("if (dj < db - 1e-9 * (db > 0 ? db : 1.0)) best = j;",
                           "if (dj > db + 1e-9 * (db > 0 ? db : 1.0)) best = j;", 0, 1, [PINS]),
    "legendre_recurrence": ("- n * p0) / (n + 1.0);", "- (n + 1.0) * p0) / (n + 1.0);", 0, 1, [PINS]),
    "legendre_norm": ("return sqrt(2.0 * j + 1.0) * p1;", "return sqrt(2.0 * j) * p1;", 0, 1, [PINS]),
    "legendre_interval": ("double s = 2.0 * t - 1.0;", "double s = t;", 0, 1, [PINS]),
    "vandermonde_transposed": ("P->V[a * nx + b2] = leg_tensor(d, P->alpha + b2 * d, P->xi + a * d);",
                               "P->V[a * nx + b2] = leg_tensor(d, P->alpha + a * d, P->xi + b2 * d);", 0, 1,
                               [PINS]),
    # tree (Sec 5.1) and block partition (Sec 5.2, eq. (admissibility))
    "split_shortest_edge": ("if (ext > best) { best = ext; a = k; }",
                            "if (best < 0.0 || ext < best) { best = ext; a = k; }", 0, 1, [PINS]),
    "split_off_median": ("long half = (m + 1) / 2;", "long half = m / 2 + 1;", 0, 1, [PINS]),
    "box_not_tight": ("if (x[k] > hi[k]) hi[k] = x[k];", "if (x[k] > hi[k]) hi[k] = x[k] + 1e-3;", 0, 1, [PINS]),
    "admissibility_eta_unsquared": ("return dist2 >= eta * eta * dm;", "return dist2 >= eta * dm;", 0, 1,
                                    [PINS, ADM]),
    "box_gap_min": ("double g = g1 > g2 ? g1 : g2;", "double g = g1 < g2 ? g1 : g2;", 0, 2, [PINS, ADM]),
    # transfer matrices, upward / coupling / downward passes, nearfield (Sec 5.2)
    "transfer_child_box": ("map_from_box(d, P->lo + pa * d, P->hi + pa * d, xc, t);",
                           "map_from_box(d, P->lo + c * d, P->hi + c * d, xc, t);", 0, 1, [PINS]),
    "m2m_transposed": ("+= Tc[a * nx + b2] * mom[(ch * nx + a) * nrhs + r];",
                       "+= Tc[b2 * nx + a] * mom[(ch * nx + a) * nrhs + r];", 0, 2, [PINS]),
    "coupling_vinv_untransposed": ("sum += W[a * nx + g] * P->Vinv[b2 * nx + g];",
                                   "sum += W[a * nx + g] * P->Vinv[g * nx + b2];", 0, 1, [PINS]),
    "coupling_nodes_swapped": ("S[a * nx + b2] = orc_kernel(P->kind, P->ell, d, xa + a * d, xb + b2 * d);",
                               "S[a * nx + b2] = orc_kernel(P->kind, P->ell, d, xa + b2 * d, xb + a * d);", 0, 1,
                               [PINS]),
    "l2l_transposed": ("+= Tc[a * nx + b2] * loc[(c * nx + b2) * nrhs + r];",
                       "+= Tc[b2 * nx + a] * loc[(c * nx + b2) * nrhs + r];", 0, 2, [PINS]),
    "near_wrong_source": ("orc_kernel(P->kind, P->ell, d, P->X + oi * d, P->X + oj * d);",
                          "orc_kernel(P->kind, P->ell, d, P->X + oi * d, P->X + oi * d);", 0, 1, [PINS]),
    "near_overwrites": ("y[oi * nrhs + r] += k * x[oj * nrhs + r];", "y[oi * nrhs + r] = k * x[oj * nrhs + r];",
                        0, 2, [PINS]),
    # CG on (K~ + lambda I) alpha = f, eq. (LGS)
    "cg_beta_inverted": ("double beta = rn / rr[c];", "double beta = rr[c] / rn;", 0, 1, [PINS]),
    "cg_ridge_dropped": ("out[i] += lambda * v[i];", "out[i] += lambda;", 0, 1, [PINS]),
    # approximate Fekete points and Lebesgue constant (Sec 5.4)
    "afp_smallest_column": ("if (s > best) best = s;", "if (best < 0.0 || s < best) best = s;", 0, 1, [AFP]),
    "halton_from_zero": ("orc_radical_inverse(j + 1, nth_prime(r++))", "orc_radical_inverse(j, nth_prime(r++))",
                         0, 1, [AFP]),
    "radical_inverse_digit": ("num = num * p + i % p;", "num = num * p + i / p;", 0, 1, [AFP]),
    "lebesgue_vinv_transposed": ("l += P->Vinv[(size_t)g * nx + a] * p[g];",
                                 "l += P->Vinv[(size_t)a * nx + g] * p[g];", 0, 1, [LEB]),
    # evaluation at new points: the same passes over a target tree
    "eval_l2l_transposed": ("+= Tc[a * nx + b2] * loc[(c * nx + b2) * nrhs + r];",
                            "+= Tc[b2 * nx + a] * loc[(c * nx + b2) * nrhs + r];", 1, 2, [EVAL]),
    "eval_near_overwrites": ("y[oi * nrhs + r] += k * x[oj * nrhs + r];",
                             "y[oi * nrhs + r] = k * x[oj * nrhs + r];", 1, 2, [EVAL]),
}


def mutate(text, frag, repl, occ, count):
    assert text.count(frag) == count, (frag, text.count(frag))
    pos = -1
    for _ in range(occ + 1):
        pos = text.index(frag, pos + 1)
    return text[:pos] + repl + text[pos + len(frag):]


def run_pins(name, text, files):
    """Compile `text` and run the pin files against it; returns (exit status, output tail)."""
    import oracle
    tmp = tempfile.mkdtemp(prefix=f"orc_{name}_")
    try:
        src, lib = os.path.join(tmp, "oracle.c"), os.path.join(tmp, "oracle.so")
        pathlib.Path(src).write_text(text)
        oracle.compile_source(src, lib)
        env = dict(os.environ, DWFMM_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
        cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-p", "no:xdist",
               "-m", "not gpu"] + [str(ROOT / "tests" / f) for f in files]
        p = subprocess.run(cmd, cwd=str(ROOT), env=env, capture_output=True, text=True, timeout=600)
        return p.returncode, (p.stdout + p.stderr)[-1500:]
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def test_every_planted_mistake_is_caught():
    """One test (so that a parallel test run computes the cases once): the unmodified copy passes
    every pin file, and each planted mistake makes its pins fail (exit status 1; a crash of the
    child, another status, is not accepted)."""
    text = SRC.read_text()
    jobs = {"unmodified": (text, ALL)}
    for name, (frag, repl, occ, count, files) in MUTANTS.items():
        jobs[name] = (mutate(text, frag, repl, occ, count), files)
    with ThreadPoolExecutor(4) as ex:
        futs = {k: ex.submit(run_pins, k, t, f) for k, (t, f) in jobs.items()}
        res = {k: f.result() for k, f in futs.items()}
    rc, out = res.pop("unmodified")
    assert rc == 0, out
    missed = {k: v for k, v in res.items() if v[0] != 1}
    assert not missed, "\n".join(f"{k}: exit {rc}\n{out}" for k, (rc, out) in missed.items())
