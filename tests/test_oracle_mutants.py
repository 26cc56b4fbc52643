"""Strength of the oracle's pins: plausible mistakes planted in a copy of the
oracle must each make a pin fail.

Every mutant below is one small edit of the kind that slips into such code (a
dropped term or factor, a wrong sign, a swapped index or operand, a wrong
constant). The edit is applied to a temporary copy of ``oracle/`` (C++ and
Python), the copy is built, and the pins named for that mutant
(``tests/test_oracle_pins.py``, selected with ``-k``) are run against the copy
in a subprocess; the mutant counts as caught when they fail. An unmutated copy
runs the same selection first and must pass, so a failure always means the
planted mistake and never the harness. Everything runs on the CPU; the
repository's own oracle is never modified.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CPP = "oracle/lbm_oracle.cpp"
PY = "oracle/__init__.py"

# (name, file, [(old, new), ...], pins selected with -k)
MUTANTS = [
    # ---- lattice, equilibrium, moments (C++)
    ("feq quadratic coefficient 4.5 -> 4", CPP, [("4.5 * cu * cu", "4.0 * cu * cu")], "equilibrium_moments"),
    ("feq |u|^2 term sign", CPP, [("- 1.5 * usq", "+ 1.5 * usq")], "equilibrium_moments"),
    ("velocity not divided by rho", CPP, [("u[a] = j[a] / rho;", "u[a] = j[a];")], "fixed_point"),
    ("D3Q19 axis and diagonal weights swapped", CPP,
     [("{1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0}", "{1.0 / 3.0, 1.0 / 36.0, 1.0 / 18.0}")], "d3q19_velocity_set"),
    ("velocity index order transposed (cz slowest)", CPP,
     [("c[k][0] = a - 1;", "c[k][0] = d - 1;"), ("c[k][2] = d - 1;", "c[k][2] = a - 1;")], "index_convention"),
    # (M020 - M200 in place of M020 - M002 spans the same shear subspace and
    # leaves the collision unchanged: not a mistake, so not listed)
    ("normal-stress difference with a sign error", CPP,
     [("M[row][i] = raw(2, 0, 0, i) - raw(0, 0, 2, i);", "M[row][i] = raw(2, 0, 0, i) + raw(0, 0, 2, i);")],
     "shear_hom_split"),
    ("off-diagonal stress put in the hom group", CPP, [("put_raw(1, 1, 0, 1);", "put_raw(1, 1, 0, 2);")],
     "shear_hom_split"),
    ("trace put in the shear group", CPP, [("group[row++] = 2;", "group[row++] = 1;")], "shear_hom_split"),
    # ---- collision (C++)
    ("stabiliser: sign of the correction", CPP,
     [("gamma = 2.0 / omega - (2.0 - 2.0 / omega) * sh / hh;", "gamma = 2.0 / omega + (2.0 - 2.0 / omega) * sh / hh;")],
     "closed_form_gamma"),
    ("stabiliser: inner product without 1/f^eq", CPP,
     [("sh += ds[i] * dh[i] / feq[i];\n      hh += dh[i] * dh[i] / feq[i];",
       "sh += ds[i] * dh[i];\n      hh += dh[i] * dh[i];")], "closed_form_gamma"),
    ("stabiliser: 2/omega replaced by 1/omega", CPP,
     [("gamma = 2.0 / omega - (2.0 - 2.0 / omega) * sh / hh;", "gamma = 1.0 / omega - (2.0 - 2.0 / omega) * sh / hh;")],
     "closed_form_gamma or bgk_special_cases"),
    ("hom rate omega*gamma instead of omega*gamma/2", CPP, [("s = omega * gamma / 2.0;", "s = omega * gamma;")],
     "bgk_special_cases"),
    ("shear rate omega/2", CPP, [("if (mb.group[r] == 1) s = omega;", "if (mb.group[r] == 1) s = omega / 2.0;")],
     "bgk_special_cases"),
    ("post-collision state adds the relaxation", CPP, [("fstar[i] = f[i] - acc;", "fstar[i] = f[i] + acc;")],
     "bgk_special_cases"),
    ("exact stabiliser: logarithm without the weight", CPP,
     [("s += -dh[i] * (std::log(fs / v.w[i]) + 1.0);", "s += -dh[i] * (std::log(fs) + 1.0);")],
     "exact_entropic_gamma"),
    ("exact stabiliser: t returned as gamma", CPP,
     [("return 2.0 * (0.5 * (lo + hi)) / omega;", "return (0.5 * (lo + hi)) / omega;")], "exact_entropic_gamma"),
    ("exact stabiliser, complex step: Newton curvature with one dh", CPP,
     [("d2H += dh[i] * dh[i] / fs;", "d2H += dh[i] / fs;")], "complex_step_through"),
    ("exact stabiliser, complex step: logarithm without the weight", CPP,
     [("dH -= dh[i] * (std::log(fs / v.w[i]) + 1.0);", "dH -= dh[i] * (std::log(fs) + 1.0);")],
     "complex_step_through"),
    ("time loop does not keep the new state", CPP, [("std::memcpy(f, tmp.data(), sizeof(T) * len);", "")],
     "streaming_is_a_permutation"),
    # ---- streaming and initial populations (C++)
    ("streaming against the velocity", CPP,
     [("int xs = (x - v.c[i][0] + n) % n;", "int xs = (x + v.c[i][0] + n) % n;")], "streaming_is_a_permutation"),
    ("streaming: y shifted by c_z", CPP,
     [("int ys = (y - v.c[i][1] + n) % n;", "int ys = (y - v.c[i][2] + n) % n;")], "streaming_is_a_permutation"),
    ("initial populations: y and z velocity swapped", CPP,
     [("double uc[3] = {u[cell], u[ncell + cell], u[2 * ncell + cell]};",
       "double uc[3] = {u[cell], u[2 * ncell + cell], u[ncell + cell]};")], "initial_populations"),
    ("initial populations: density 1 + |u|^2", CPP,
     [("equilibrium<Q, double>(1.0, uc, f + cell * Q);",
       "equilibrium<Q, double>(1.0 + uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2], uc, f + cell * Q);")],
     "initial_populations or initial_kinetic_energy"),
    # ---- parameters (Python)
    ("omega: 2 nu replaced by nu", PY, [("return 2.0 * cs2 / (2.0 * nu + cs2)", "return 2.0 * cs2 / (nu + cs2)")],
     "unit_conversion"),
    ("lattice length n/pi instead of n/(2 pi)", PY,
     [("return u0 * (n / (2.0 * math.pi)) / re", "return u0 * (n / math.pi) / re")], "lattice_viscosity"),
    ("table time step without dx", PY, [("dt = dx * u_lu", "dt = u_lu")], "unit_conversion"),
    ("Mach number taken relative to 1 instead of c_s", PY, [("u_lu = ma * math.sqrt(1.0 / 3.0)", "u_lu = ma")],
     "unit_conversion"),
    # ---- initial data (Python)
    ("grid spacing 2 pi/(n-1)", PY, [("x = 2.0 * math.pi * np.arange(n) / n", "x = 2.0 * math.pi * np.arange(n) / (n - 1)")],
     "taylor_green_field"),
    ("Taylor-Green: sign of the y component", PY,
     [("-np.cos(X) * np.sin(Y) * np.cos(Z)", "np.cos(X) * np.sin(Y) * np.cos(Z)")], "taylor_green_field"),
    ("perturbation: coefficient index order", PY,
     [("y[8 * al + 4 * i + 2 * j + k]", "y[8 * al + i + 2 * j + 4 * k]")], "leray_projection"),
    ("perturbation: sine and cosine swapped", PY, [("a = (np.sin, np.cos)", "a = (np.cos, np.sin)")],
     "leray_projection"),
    ("perturbation: wavenumber 1 instead of 2", PY,
     [("a[i](2 * X) * a[j](2 * Y) * a[k](2 * Z)", "a[i](X) * a[j](Y) * a[k](Z)")], "leray_projection"),
    ("perturbation: factor 1/8 dropped", PY, [("return s / 8.0", "return s")], "initial_kinetic_energy"),
    ("Leray projection: sign of the gradient removal", PY,
     [("vh[a] - K[a] * div / k2", "vh[a] + K[a] * div / k2")], "leray_projection"),
    # ---- moments and reductions (Python)
    ("moments: velocity not divided by rho", PY, [("u = (j / rho[:, None]).T", "u = j.T")], "moments_of"),
    ("reductions: x and y momentum swapped", PY,
     [("j[:, 0].sum(), j[:, 1].sum(), j[:, 2].sum()", "j[:, 1].sum(), j[:, 0].sum(), j[:, 2].sum()")], "moments_of"),
    ("complex step divided by 2h", PY, [("grad[p] = kinetic_energy(u).imag / h", "grad[p] = kinetic_energy(u).imag / (2 * h)")],
     "complex_step"),
    ("kinetic energy without the 1/2", PY, [("return 0.5 * np.mean(u[0] * u[0]", "return np.mean(u[0] * u[0]")],
     "initial_kinetic_energy"),
    # ---- observables (Python)
    ("spectrum: shells by floor instead of rounding", PY,
     [("shell = np.floor(np.sqrt(kmag2) + 0.5)", "shell = np.floor(np.sqrt(kmag2))")], "spectrum"),
    ("spectrum: 1/2 dropped", PY, [("0.5 * kmag2[sel] * phi[sel]", "kmag2[sel] * phi[sel]")], "spectrum"),
    ("spectrum: coefficients not normalised by N^3", PY,
     [("uh = np.stack([np.fft.fftn(u[a]) / n ** 3 for a in range(3)])",
       "uh = np.stack([np.fft.fftn(u[a]) / n ** 2 for a in range(3)])")], "spectrum"),
    ("structure function: factor 2 dropped", PY,
     [("S[r - 1] = np.mean(2.0 * (R[0, 0, 0] - R[sel]))", "S[r - 1] = np.mean(R[0, 0, 0] - R[sel])")],
     "structure_function"),
    ("structure function: shells by floor", PY,
     [("rr = np.floor(np.sqrt(HX ** 2 + HY ** 2 + HZ ** 2) + 0.5)", "rr = np.floor(np.sqrt(HX ** 2 + HY ** 2 + HZ ** 2))")],
     "structure_function"),
    ("autocorrelation normalised by N^6", PY, [("return np.fft.ifftn(psd).real / n ** 3", "return np.fft.ifftn(psd).real / n ** 6")],
     "structure_function"),
    ("W1 without sorting the second law", PY,
     [("b = np.sort(np.asarray(b, dtype=np.float64))", "b = np.asarray(b, dtype=np.float64)")], "wasserstein"),
    ("sample error normalised by the sample, not the reference", PY,
     [("den = sum(abs(b[s, c, k]) for k in range(g))", "den = sum(abs(a[s, c, k]) for k in range(g))")],
     "sample_error"),
    ("sample error: vector term overwritten, not accumulated", PY,
     [("out[3] += np.float64(num) / np.float64(den)", "out[3] = np.float64(num) / np.float64(den)")], "sample_error"),
    ("order of convergence: axes swapped", PY,
     [("return float(np.polyfit(np.log(np.asarray(ns, dtype=np.float64)),\n"
       "                            np.log(np.asarray(ds, dtype=np.float64)), 1)[0])",
       "return float(np.polyfit(np.log(np.asarray(ds, dtype=np.float64)),\n"
       "                            np.log(np.asarray(ns, dtype=np.float64)), 1)[0])")], "eoc_slope"),
    ("standard deviation with 1/M", PY, [("/ (m - 1))", "/ m)")], "ensemble_mean_std"),
    ("compensated spectrum: exponent 3/5", PY, [("kap ** (5.0 / 3.0)", "kap ** (3.0 / 5.0)")], "compensation"),
    ("compensated spectrum: Kolmogorov constant 1.6", PY,
     [("KOLMOGOROV_CONSTANT = 1.5", "KOLMOGOROV_CONSTANT = 1.6")], "compensation"),
    ("compensated structure function: lag in lattice units", PY,
     [("r = (j + 1) * 2.0 * math.pi / n", "r = (j + 1)")], "compensation"),
    # ---- dissipation rate and Kolmogorov length (Python)
    ("decay rate: sign of the derivative", PY,
     [("out[k] = -(e[hi] - e[lo]) / (t[hi] - t[lo])", "out[k] = (e[hi] - e[lo]) / (t[hi] - t[lo])")], "decay_rate"),
    ("decay rate: centred difference over one interval", PY,
     [("out[k] = -(e[hi] - e[lo]) / (t[hi] - t[lo])", "out[k] = -(e[hi] - e[lo]) / (t[hi] - t[k] + 1e-300)")],
     "decay_rate"),
    ("dissipation from spectra: lattice units kept", PY,
     [("total[k, s] = sum(ek[k, s, kap] for kap in range(ek.shape[2])) / u0[s] ** 2",
       "total[k, s] = sum(ek[k, s, kap] for kap in range(ek.shape[2]))")], "dissipation_from_spectra"),
    ("dissipation from spectra: shell weight dropped (kinetic energy instead)", PY,
     [("total[k, s] = sum(ek[k, s, kap] for kap in range(ek.shape[2])) / u0[s] ** 2",
       "total[k, s] = sum(ek[k, s, kap] for kap in range(ek.shape[2])) / u0[s] ** 2 / (4 * math.pi * 3 / 62)")],
     "dissipation_from_spectra"),
    ("dissipation definition: k_z dropped from |k|^2", PY,
     [("k2 = KX ** 2 + KY ** 2 + KZ ** 2\n    phi = sum(", "k2 = KX ** 2 + KY ** 2\n    phi = sum(")],
     "dissipation_definition"),
    ("dissipation definition: coefficients without the 1/N^3 of eq. (dftCoeff)", PY,
     [("phi = sum(np.abs(np.fft.fftn(u[a] / u0) / n ** 3) ** 2 for a in range(3))",
       "phi = sum(np.abs(np.fft.fftn(u[a] / u0) / n ** 2) ** 2 for a in range(3))")], "dissipation_definition"),
    ("Kolmogorov length: exponent 1/3", PY, [("return (eps ** 3 / mean) ** 0.25", "return (eps ** 3 / mean) ** (1.0 / 3.0)")],
     "kolmogorov_length"),
    ("Kolmogorov length: sum over samples instead of the mean", PY,
     [("mean = np.sum(d, axis=-1) / d.shape[-1]", "mean = np.sum(d, axis=-1)")], "kolmogorov_length"),
]

PIN_FILE = "tests/test_oracle_pins.py"


def _copy_tree(dst):
    """The files a pin run needs, copied from the repository."""
    for d in ("oracle", "mc_inputs"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d),
                        ignore=shutil.ignore_patterns("__pycache__", "*.so", "*.tmp"))
    os.makedirs(os.path.join(dst, "tests"))
    for f in ("conftest.py", "test_oracle_pins.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(dst, "tests", f))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(dst, "tests", "golden"),
                    ignore=shutil.ignore_patterns("__pycache__", "*.npz"))


def _build(d):
    src = os.path.join(d, "oracle", "lbm_oracle.cpp")
    lib = os.path.join(d, "oracle", "liboracle.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", lib, src], check=True,
                   capture_output=True, text=True)


def _run_pins(d, expr):
    env = {k: v for k, v in os.environ.items() if k != "PYTHONPATH"}
    env.update(PYTHONDONTWRITEBYTECODE="1", OMP_NUM_THREADS="1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu and not slow",
           "-k", expr, PIN_FILE]
    p = subprocess.run(cmd, cwd=d, env=env, capture_output=True, text=True, timeout=600)
    return p.returncode, p.stdout[-3000:] + p.stderr[-2000:]


def _mutant(base, work, k):
    name, path, edits, expr = MUTANTS[k]
    d = os.path.join(work, f"m{k:02d}")
    shutil.copytree(base, d)
    fp = os.path.join(d, path)
    with open(fp) as fh:
        text = fh.read()
    for old, new in edits:
        if text.count(old) != 1:
            return ("harness", f"edit target occurs {text.count(old)} times: {old!r}")
        text = text.replace(old, new)
    with open(fp, "w") as fh:
        fh.write(text)
    if path == CPP:
        _build(d)
    else:
        shutil.copy(os.path.join(base, "oracle", "liboracle.so"), os.path.join(d, "oracle", "liboracle.so"))
    rc, out = _run_pins(d, expr)
    shutil.rmtree(d, ignore_errors=True)
    return ("caught" if rc == 1 else ("survived" if rc == 0 else "harness"), out)


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    work = str(tmp_path_factory.mktemp("oracle_mutants"))
    base = os.path.join(work, "base")
    _copy_tree(base)
    _build(base)
    # control: the unmutated copy passes every selection used below
    union = " or ".join(sorted({m[3] for m in MUTANTS}))
    rc, out = _run_pins(base, union)
    assert rc == 0, "the unmutated oracle copy fails its pins:\n" + out
    workers = max(1, min(8, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        res = list(ex.map(lambda k: _mutant(base, work, k), range(len(MUTANTS))))
    return res


@pytest.mark.parametrize("k", range(len(MUTANTS)), ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(outcomes, k):
    status, out = outcomes[k]
    name, _, _, expr = MUTANTS[k]
    assert status == "caught", f"mutant '{name}' {status} the pins selected by -k '{expr}':\n{out}"
