"""CPU checks of the HIP library: it loads, exports every entry point the
header declares, and its host-side logic (filter coefficients, closed-form
filter, plan and order K) agrees with the oracle.  No GPU compute calls."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads as wl
from oracle import filter as flt
from oracle import lanczos, models, polfed

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polfed.h")


@pytest.fixture(scope="module")
def pk():
    import paper_2605_10191_amd as pk
    pk.load_library()
    return pk


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(polfed_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol(pk):
    lib = pk.load_library()
    names = declared_symbols()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares a signature for every status-returning call
    assert set(pk.SIGNATURES) | {"polfed_version", "polfed_last_error"} == set(names)


def struct_fields(name):
    """(field, C type) of a typedef'd struct of the header, in order."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + ";", txt).group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            typ, names = decl.split(None, 1)
            out += [(n.strip(), typ) for n in names.split(",")]
    return out


def test_binding_structs_and_constants_match_the_header(pk):
    ctypes_of = {"double": ctypes.c_double, "int": ctypes.c_int}
    for cname, cls in (("polfed_report", pk.Report), ("polfed_params", pk.Params),
                       ("polfed_plan", pk.Plan)):
        want = [(n, ctypes_of[t]) for n, t in struct_fields(cname)]
        got = [(n.rstrip("_"), t) for n, t in cls._fields_]
        assert got == want, cname
    txt = open(HEADER).read()
    for cname, val in (("POLFED_FP64", pk.FP64), ("POLFED_FP32", pk.FP32),
                       ("POLFED_PRECISION_AUTO", pk.AUTO)):
        assert int(re.search(cname + r"\s*=\s*(\d+)", txt).group(1)) == val


def test_version_and_basis_dim(pk):
    assert pk.load_library().polfed_version() >= 10000
    for L, N in [(12, 6), (20, 10), (24, 12), (26, 13), (32, 16), (5, 0)]:
        assert pk.basis_dim(L, N) == math.comb(L, N)


def test_invalid_arguments_are_reported(pk):
    with pytest.raises(pk.PolfedError) as e:
        pk.make_plan(100, 1.0, -1.0, 1e-3, 0.0, 0.0, 1.0, 10)
    assert e.value.code == -1 and "E_min" in str(e.value)
    with pytest.raises(pk.PolfedError):
        pk.filter_coefficients(0.2, -1)
    with pytest.raises(pk.PolfedError):
        pk.basis_dim(40, 3)


def test_no_device_is_an_error_not_a_crash(pk):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    code = pk.load_library().polfed_create(0, None, ctypes.byref(h))
    assert code == -7


@pytest.mark.parametrize("lam_t,K", [(0.0, 10), (0.31, 281), (-0.62, 2000),
                                     (0.5, 14000)])
def test_filter_coefficients_match_oracle(pk, lam_t, K):
    a = pk.filter_coefficients(lam_t, K)
    ref = flt.coefficients(lam_t, K)
    # the oracle runs the Chebyshev recurrence, the library cos(n phi):
    # rounding differences grow at most linearly in n
    assert np.max(np.abs(a - ref)) <= 4e-16 * K * np.max(np.abs(ref)) + 1e-18


@pytest.mark.parametrize("lam_t,K", [(0.0, 10), (0.31, 281), (-0.62, 700)])
def test_closed_form_filter_matches_direct_sum(pk, lam_t, K):
    x = np.concatenate([np.linspace(-1, 1, 401), [lam_t]])
    got = pk.filter_value(lam_t, K, x)
    ref = flt.filter_value(x, lam_t, K)
    assert np.max(np.abs(got - ref)) < 1e-11
    assert abs(got[-1] - 1.0) < 1e-13


def test_plan_matches_oracle_on_xxz_l12():
    import paper_2605_10191_amd as pk
    H, _ = models.xxz(12, 6, 1.0, 1.0, wl.xxz_fields(12, 1.0, 0))
    E_min, E_max = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("normalized", 0.5, E_min, E_max)
    n_window = 20 + polfed.buffer_size(20)
    ref = polfed.plan(H, lam, n_window, E_min, E_max)
    tr1, tr2 = flt.trace_moments(H)
    p = pk.make_plan(H.shape[0], E_min, E_max, 1e-3, lam, tr1, tr2, n_window)
    for f in ("E_c", "dE", "lam_t", "mu_t", "Gamma_t", "rho", "delta"):
        g = getattr(p, "lambda_t" if f == "lam_t" else f)
        assert abs(g - ref[f]) <= 1e-12 * max(1.0, abs(ref[f])), f
    assert p.K == ref["K"]


def test_order_K_matches_oracle_bisection(pk):
    """Integer decision taken in FP64 on both sides; allow a difference only
    where the oracle's own predicate sits within rounding of the cutoff."""
    rng = np.random.default_rng(7)
    mism = 0
    for _ in range(40):
        lam_t = rng.uniform(-0.7, 0.7)
        p = _lib_plan(pk, lam_t, 10 ** rng.uniform(-3.5, -1.5))
        delta, K_lib = p.delta, p.K
        K_ref = flt.choose_K(lam_t, delta)
        if K_lib != K_ref:
            mism += 1
            pts = np.array([lam_t - delta, lam_t + delta])
            edge = np.min(flt.filter_value(pts, lam_t, max(K_lib, K_ref)))
            assert abs(edge - flt.OMEGA_DEFAULT) < 1e-10
    assert mism <= 1


def _lib_plan(pk, lam_t, delta):
    """Library plan for (about) a given window half-width: choose the
    Gaussian so that rho(lambda~) = 1/(2 delta) with D = 1 and n_window = 1
    (mu = lambda~, Gamma = 1/(2 delta sqrt(2 pi)) in rescaled units)."""
    Gamma = 2 * delta / math.sqrt(2 * math.pi)
    # D / (sqrt(2 pi) Gamma) = 1 / (2 delta)  ->  D = 1
    tr1 = lam_t
    tr2 = lam_t ** 2 + Gamma ** 2
    p = pk.make_plan(1, -1.0, 1.0, 0.0, lam_t, tr1, tr2, 1)
    assert abs(p.delta - delta) < 1e-9 * delta
    return p


@pytest.mark.parametrize("K,theta", [(1, 0.3), (2, -0.7), (3, 0.11), (60, 0.25),
                                     (281, -0.4), (1500, 0.02)])
def test_filter_quotient_is_the_divided_difference(pk, K, theta):
    """Q(x) (x - theta) = p(x) - p(theta), checked with NumPy's Chebyshev
    series at points away from theta, and Q(theta) = p'(theta)."""
    from numpy.polynomial import chebyshev as C
    rng = np.random.default_rng(K)
    a = rng.standard_normal(K + 1) / (K + 1)
    q, p_th = pk.filter_quotient(a, theta)
    assert q.shape == (K,)
    assert abs(p_th - C.chebval(theta, a)) <= 1e-13
    x = rng.uniform(-1, 1, 200)
    x = x[np.abs(x - theta) > 0.05]
    lhs = C.chebval(x, q) * (x - theta)
    rhs = C.chebval(x, a) - C.chebval(theta, a)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * max(1.0, np.max(np.abs(rhs))) * K
    deriv = C.chebval(theta, C.chebder(a))
    assert abs(C.chebval(theta, q) - deriv) <= 1e-11 * max(1.0, abs(deriv)) * K


def test_filter_quotient_order_zero(pk):
    q, p_th = pk.filter_quotient([0.7], 0.2)
    assert q.shape == (0,) and p_th == 0.7


def test_kpm_density_matches_oracle(pk):
    """The host KPM density (Clenshaw sum) against the oracle's cosine form."""
    from oracle import kpm
    mu = np.random.default_rng(2).standard_normal(70) * np.exp(-0.05 * np.arange(70))
    mu[0] = 50.0
    x = np.linspace(-0.97, 0.97, 301)
    got = pk.kpm_density(mu, x)
    ref = kpm.density(mu, x)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_kpm_density_rejects_points_outside_the_interval(pk):
    with pytest.raises(pk.PolfedError):
        pk.kpm_density(np.ones(10), [0.5, 1.0])
    with pytest.raises(pk.PolfedError):
        pk.kpm_density(np.ones(10), [-1.5])


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; asked for more it says so and exits
    before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_product_path_is_independent_of_the_oracle():
    """The library package neither imports nor links the oracle, and the HIP
    sources include nothing from it; bench.py reaches it only in its CPU
    baseline leg."""
    import ast
    pkg = os.path.join(ROOT, "paper_2605_10191_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            path = os.path.join(dirpath, f)
            if f.endswith(".py"):
                tree = ast.parse(open(path).read())
                for node in ast.walk(tree):
                    if isinstance(node, ast.Import):
                        assert not any(a.name.split(".")[0] == "oracle" for a in node.names), path
                    if isinstance(node, ast.ImportFrom):
                        assert (node.module or "").split(".")[0] != "oracle", path
            elif f.endswith((".hip", ".cpp", ".hpp", ".h")):
                assert "oracle" not in open(path).read(), path
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    users = {fn.name for fn in ast.walk(tree) if isinstance(fn, ast.FunctionDef)
             for node in ast.walk(fn)
             if isinstance(node, ast.ImportFrom) and (node.module or "").startswith("oracle")}
    assert users == {"cpu_baseline"}
