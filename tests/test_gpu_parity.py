"""GPU parity: every call of the C ABI against the CPU oracle on the same
seeded inputs.  Integer work bit-exact; FP64 within the stated tolerances;
eigenpairs within 1e-10 relative energy and 1e-8 residual."""
import functools
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import basis, dense, lanczos, models, polfed
from oracle import filter as flt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_10191_amd as pk
    pk.load_library()
    return pk


@pytest.fixture(scope="module")
def ctx(pk):
    c = pk.Context(0)
    yield c
    c.sync()


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@functools.lru_cache(maxsize=None)
def xxz_case(L, N, W, seed, periodic=True, J=1.0, Delta=1.0):
    h = wl.xxz_fields(L, W, seed)
    H, st = models.xxz(L, N, J, Delta, h, periodic)
    return h, H, st


@functools.lru_cache(maxsize=None)
def tv_case(L, N, seed, periodic=True):
    eps = wl.tv_onsite(L, seed)
    H, st = models.tv(L, N, 1.0, 1.0, eps, periodic)
    return eps, H, st


@functools.lru_cache(maxsize=None)
def qsun_case(N, L, seed, alpha=0.75):
    q = wl.qsun_draws(N, L, seed)
    H = models.qsun(N, L, q["A"], 1.0, 1.0, alpha, q["u"], q["n_of_j"], q["h"])
    return q, H


def make_op(pk, ctx, kind, *args):
    if kind == "xxz":
        L, N, W, seed, periodic = args
        h, H, _ = xxz_case(L, N, W, seed, periodic)
        return pk.Operator.xxz(ctx, L, N, 1.0, 1.0, h, periodic), H
    if kind == "tv":
        L, N, seed, periodic = args
        eps, H, _ = tv_case(L, N, seed, periodic)
        return pk.Operator.tv(ctx, L, N, 1.0, 1.0, eps, periodic), H
    if kind == "qsun":
        N, L, seed = args
        q, H = qsun_case(N, L, seed)
        return pk.Operator.qsun(ctx, N, L, q["A"], 1.0, 1.0, 0.75, q["u"],
                                q["n_of_j"], q["h"]), H
    raise ValueError(kind)


OPS = [("xxz", 12, 6, 1.0, 0, True), ("xxz", 13, 5, 3.0, 1, True),
       ("xxz", 11, 4, 2.0, 2, False), ("xxz", 16, 8, 3.0, 3, True),
       ("tv", 12, 6, 1, True), ("tv", 11, 5, 2, True), ("tv", 10, 4, 3, False),
       ("qsun", 3, 7, 0), ("qsun", 2, 9, 1)]


# ----------------------------------------------------------------- basis ----

@pytest.mark.parametrize("L,N", [(1, 1), (6, 3), (12, 6), (13, 4), (20, 10),
                                 (24, 12)])
def test_basis_enumerate_rank_unrank_bit_exact(pk, ctx, L, N):
    say(f"basis L={L} N={N}")
    ref = basis.sector_states(L, N)
    st = ctx.basis_enumerate(L, N)
    got = host(st).astype(np.int64) & 0xFFFFFFFF
    assert np.array_equal(got, ref)
    r = host(ctx.basis_rank(L, N, st))
    assert np.array_equal(r, np.arange(len(ref)))
    rng = np.random.default_rng(L)
    pick = rng.integers(0, len(ref), min(len(ref), 5000))
    back = host(ctx.basis_unrank(L, N, dev(pick, torch.int64)))
    assert np.array_equal(back.astype(np.int64) & 0xFFFFFFFF, ref[pick])


def test_basis_invalid_inputs(pk, ctx):
    say("basis invalid")
    bad = dev(np.array([0b111, 0b1, 1 << 12 | 0b11111], dtype=np.int32), torch.int32)
    r = host(ctx.basis_rank(12, 6, bad))
    assert np.all(r == -1)
    out = host(ctx.basis_unrank(12, 6, dev(np.array([-1, 924, 0]), torch.int64)))
    out = out.astype(np.int64) & 0xFFFFFFFF
    assert out[0] == 0xFFFFFFFF and out[1] == 0xFFFFFFFF
    assert out[2] == 0b111111
    with pytest.raises(pk.PolfedError):
        ctx.basis_enumerate(33, 3)


# ------------------------------------------------------------- operators ----

@pytest.mark.parametrize("case", OPS, ids=lambda c: "-".join(map(str, c)))
def test_operator_apply_matches_oracle(pk, ctx, case):
    say(f"apply {case}")
    op, H = make_op(pk, ctx, *case)
    x = np.random.default_rng(1).standard_normal(op.D)
    y = host(op.apply(dev(x)))
    ref = H @ x
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("case", OPS, ids=lambda c: "-".join(map(str, c)))
def test_materialized_csr_equals_oracle_matrix(pk, ctx, case):
    say(f"csr {case}")
    op, H = make_op(pk, ctx, *case)
    op.materialize_csr()
    rp, col, val, dg = (host(t) for t in op.export_csr())
    Href = H.tocsr().copy()
    Href.sort_indices()
    off = Href - __import__("scipy.sparse", fromlist=["diags"]).diags(Href.diagonal())
    off.eliminate_zeros()
    off.sort_indices()
    assert np.array_equal(rp, off.indptr)
    assert np.array_equal(col, off.indices)
    assert np.max(np.abs(val - off.data)) <= 1e-15 * max(1.0, np.max(np.abs(off.data)))
    assert np.max(np.abs(dg - Href.diagonal())) <= 1e-13 * max(1.0, np.max(np.abs(dg)))
    # the CSR path of the step kernel
    op.set_storage(pk.CSR)
    x = np.random.default_rng(2).standard_normal(op.D)
    y = host(op.apply(dev(x)))
    assert np.max(np.abs(y - H @ x)) <= 1e-13 * np.max(np.abs(H @ x))


def test_generic_csr_operator_with_long_rows(pk, ctx):
    """A generic CSR with a dense row longer than the LDS stage."""
    say("generic csr")
    rng = np.random.default_rng(5)
    D = 5000
    A = __import__("scipy.sparse", fromlist=["random"]).random(
        D, D, density=0.002, random_state=5, format="csr")
    A = A + A.T
    dense_row = np.zeros(D)
    dense_row[:] = rng.standard_normal(D)
    import scipy.sparse as sp
    B = sp.lil_matrix((D, D))
    B[7, :] = dense_row
    B[:, 7] = dense_row[:, None]
    A = (A + B.tocsr()).tocsr()
    A.sort_indices()
    op = pk.Operator.csr(ctx, D, A.indptr, A.indices, A.data)
    x = rng.standard_normal(D)
    y = host(op.apply(dev(x)))
    assert np.max(np.abs(y - A @ x)) <= 1e-12 * np.max(np.abs(A @ x))


@pytest.mark.parametrize("case", OPS[:6], ids=lambda c: "-".join(map(str, c)))
def test_trace_moments_match_oracle(pk, ctx, case):
    say(f"moments {case}")
    op, H = make_op(pk, ctx, *case)
    t1, t2 = op.moments()
    r1, r2 = flt.trace_moments(H)
    assert abs(t1 - r1) <= 1e-12 * max(1, abs(r1))
    assert abs(t2 - r2) <= 1e-12 * max(1, abs(r2))


def test_large_chain_sampled_rows(pk, ctx):
    """XXZ L=24 (D = 2,704,156) at full size: sampled rows of H x against the
    oracle's row-by-row evaluation of eq. (xxz)."""
    say("L=24 sampled rows")
    L, N = 24, 12
    h = wl.xxz_fields(L, 3.0, 0)
    op = pk.Operator.xxz(ctx, L, N, 1.0, 1.0, h, True)
    st = basis.sector_states(L, N)
    x = np.random.default_rng(3).standard_normal(op.D)
    y = host(op.apply(dev(x)))
    rows = np.unique(np.concatenate([
        np.random.default_rng(4).integers(0, op.D, 4000),
        np.arange(64), np.arange(op.D - 64, op.D)]))
    ref = models.xxz_rows_apply(L, N, 1.0, 1.0, h, True, st, rows, x)
    assert np.max(np.abs(y[rows] - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("L,periodic", [(22, True), (23, True), (24, True), (23, False),
                                        (24, False)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", list(range(10)))
def test_long_chain_clenshaw_step_all_rows(pk, ctx, L, periodic, prec, variant):
    """Full-size Clenshaw steps of long chains, periodic and open, with each
    step kernel (the segment kernel; the tile kernels with 8/4 (L = 22),
    16/8/4 (L = 23) and 32/16/8 (L = 24) high parts per tile; the paired-row
    and half-segment kernels; the staged-tile kernels whose tiles wrap
    around the periodic bond): every row of a v + 2 H~ b1 - b2 against the
    oracle's CSR of eq. (xxz)."""
    say(f"L={L} periodic={periodic} clenshaw step {prec} variant {variant}")
    N = L // 2
    h, H, _ = xxz_case(L, N, 3.0, 1, periodic)
    op = pk.Operator.xxz(ctx, L, N, 1.0, 1.0, h, periodic)
    p = pk.FP64 if prec == "fp64" else pk.FP32
    if variant == 5 and L == 22:
        # no tile of a quarter size at L = 22 (the largest tile has 2 bits)
        with pytest.raises(pk.PolfedError):
            op.set_kernel(p, variant)
        return
    if variant == 9 and not _has_variant(pk, op, p, variant):
        return  # two buffers of the largest tile do not fit the LDS
    assert op.set_kernel(pk.FP64 if prec == "fp64" else pk.FP32, variant) == variant
    rng = np.random.default_rng(5)
    v, b1, b2 = (rng.standard_normal(op.D) for _ in range(3))
    dt = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":  # the reference sees the same rounded inputs
        v, b1, b2 = (x.astype(np.float32).astype(np.float64) for x in (v, b1, b2))
    E_c, dE, a_i = 0.4, 23.0, 0.0173
    tb2 = dev(b2, dt)
    pk.clenshaw_step(op, E_c, dE, a_i, dev(v, dt), dev(b1, dt), tb2,
                     pk.FP64 if prec == "fp64" else pk.FP32)
    got = host(tb2).astype(np.float64)
    ref = _ref_step(H, E_c, dE, a_i, v, b1, b2, False)
    tol = 1e-13 if prec == "fp64" else 3e-6
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("L,N,periodic", [(24, 12, True), (26, 13, True), (25, 12, False)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", list(range(10)))
def test_tv_long_chain_clenshaw_step(pk, ctx, L, N, periodic, prec, variant):
    """Full-size t-V steps with every step kernel.  N = 12 makes the periodic
    hop's Jordan-Wigner sign -1, N = 13 (the L = 26 configuration) +1.  Every
    row at L = 24 against the oracle's CSR; at L = 26 (D = 10,400,600) and
    the open L = 25 chain, 6,000 random rows and the first and last 300
    against the oracle's row-by-row evaluation (models.tv_rows_apply, pinned
    on every row of smaller chains)."""
    say(f"t-V L={L} N={N} periodic={periodic} step {prec} variant {variant}")
    eps = wl.tv_onsite(L, 2)
    op = pk.Operator.tv(ctx, L, N, 1.0, 1.0, eps, periodic)
    p = pk.FP64 if prec == "fp64" else pk.FP32
    if variant == 9 and not _has_variant(pk, op, p, variant):
        return  # two buffers of the largest tile do not fit the LDS
    assert op.set_kernel(p, variant) == variant
    rng = np.random.default_rng(6)
    v, b1, b2 = (rng.standard_normal(op.D) for _ in range(3))
    dt = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        v, b1, b2 = (x.astype(np.float32).astype(np.float64) for x in (v, b1, b2))
    E_c, dE, a_i = -0.3, 31.0, 0.021
    tb2 = dev(b2, dt)
    pk.clenshaw_step(op, E_c, dE, a_i, dev(v, dt), dev(b1, dt), tb2, p)
    got = host(tb2).astype(np.float64)
    tol = 1e-13 if prec == "fp64" else 3e-6
    if L == 24:
        _, H, _ = tv_case(L, N, 2, periodic)
        ref = _ref_step(H, E_c, dE, a_i, v, b1, b2, False)
        assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))
        return
    st = _sector(L, N)
    rows = np.unique(np.concatenate([rng.integers(0, op.D, 6000), np.arange(300),
                                     np.arange(op.D - 300, op.D)]))
    Hb = models.tv_rows_apply(L, N, 1.0, 1.0, eps, periodic, st, rows, b1)
    ref = a_i * v[rows] + 2.0 * (Hb - E_c * b1[rows]) / dE - b2[rows]
    assert np.max(np.abs(got[rows] - ref)) <= tol * np.max(np.abs(ref))


def _has_variant(pk, op, prec, variant):
    """Whether the library offers this step-kernel variant for op."""
    try:
        op.set_kernel(prec, variant)
    except pk.PolfedError as e:
        assert "staged-tile" in str(e)
        return False
    return True


@functools.lru_cache(maxsize=2)
def _sector(L, N):
    return basis.sector_states(L, N)


# ----------------------------------------------------------------- filter ----

def _ref_step(H, E_c, dE, a_i, v, b1, b2, final):
    f = 0.5 if final else 1.0
    return a_i * v + f * 2.0 * (H @ b1 - E_c * b1) / dE - b2


@pytest.mark.parametrize("case", [OPS[0], OPS[2], OPS[4], OPS[7]],
                         ids=lambda c: "-".join(map(str, c)))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("final", [False, True])
def test_clenshaw_step_matches_oracle(pk, ctx, case, prec, final):
    say(f"step {case} {prec} final={final}")
    op, H = make_op(pk, ctx, *case)
    rng = np.random.default_rng(9)
    v, b1, b2 = (rng.standard_normal(op.D) for _ in range(3))
    E_c, dE, a_i = 0.3, 7.5, 0.0123
    ref = _ref_step(H, E_c, dE, a_i, v, b1, b2, final)
    dt = torch.float64 if prec == "fp64" else torch.float32
    tv_, tb1, tb2 = dev(v, dt), dev(b1, dt), dev(b2, dt)
    pk.clenshaw_step(op, E_c, dE, a_i, tv_, tb1, tb2,
                     pk.FP64 if prec == "fp64" else pk.FP32, final)
    got = host(tb2).astype(np.float64)
    tol = 1e-14 if prec == "fp64" else 2e-6
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


CHAIN_OPS = [c for c in OPS if c[0] in ("xxz", "tv")]


@pytest.mark.parametrize("case", CHAIN_OPS, ids=lambda c: "-".join(map(str, c)))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", [0, 3, 4])
def test_chain_step_variants_match_oracle(pk, ctx, case, prec, variant):
    """Every row of a Clenshaw step with the segment kernel and the paired-row
    kernel (odd segment lengths, ragged blocks, open and periodic chains)."""
    say(f"chain step variant {variant} {case} {prec}")
    op, H = make_op(pk, ctx, *case)
    p = pk.FP64 if prec == "fp64" else pk.FP32
    assert op.set_kernel(p, variant) == variant
    rng = np.random.default_rng(17)
    v, b1, b2 = (rng.standard_normal(op.D) for _ in range(3))
    dt = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        v, b1, b2 = (x.astype(np.float32).astype(np.float64) for x in (v, b1, b2))
    E_c, dE, a_i = -0.2, 9.0, 0.031
    for final in (False, True):
        tb2 = dev(b2, dt)
        pk.clenshaw_step(op, E_c, dE, a_i, dev(v, dt), dev(b1, dt), tb2, p, final)
        ref = _ref_step(H, E_c, dE, a_i, v, b1, b2, final)
        got = host(tb2).astype(np.float64)
        tol = 1e-14 if prec == "fp64" else 2e-6
        assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


def _filter_tol(K, prec):
    # forward error of the Chebyshev Clenshaw sum grows at most linearly in K
    eps = 2.2e-16 if prec == "fp64" else 1.2e-7
    return 8 * (K + 1) * eps


@pytest.mark.parametrize("case,K", [(OPS[0], 281), (OPS[3], 1500), (OPS[4], 400),
                                    (OPS[7], 600), (OPS[2], 0), (OPS[2], 1),
                                    (OPS[2], 2)],
                         ids=lambda c: "-".join(map(str, c)) if isinstance(c, tuple) else str(c))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_filter_apply_matches_oracle(pk, ctx, case, K, prec):
    say(f"filter {case} K={K} {prec}")
    op, H = make_op(pk, ctx, *case)
    E_min, E_max = lanczos.spectral_extremes(H)
    E_c, dE = flt.rescale(*lanczos.padded_bounds(E_min, E_max, 1e-3))
    lam_t = 0.13
    a = flt.coefficients(lam_t, K)
    v = wl.start_vector(op.D, 3)
    ref = flt.apply_filter(H, E_c, dE, a, v)
    dt = torch.float64 if prec == "fp64" else torch.float32
    w = pk.filter_apply(op, E_c, dE, a, dev(v, dt),
                        pk.FP64 if prec == "fp64" else pk.FP32)
    got = host(w).astype(np.float64)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    err_el = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say(f"   rel err {err:.2e}, element-wise {err_el:.2e} (tol {_filter_tol(K, prec):.1e})")
    assert err <= _filter_tol(K, prec)
    assert err_el <= _filter_tol(K, prec)


def test_filter_on_diagonal_operator_closed_form(pk, ctx):
    """H = diag(E): P(H~) v = P(E~_i) v_i with the Dirichlet closed form."""
    say("diagonal closed form")
    rng = np.random.default_rng(11)
    D = 3000
    E = rng.uniform(-4.0, 6.0, D)
    op = pk.Operator.csr(ctx, D, np.arange(D + 1), np.arange(D), E)
    E_c, dE = flt.rescale(-4.0001, 6.0001)
    lam_t, K = -0.27, 900
    a = flt.coefficients(lam_t, K)
    v = rng.standard_normal(D)
    got = host(pk.filter_apply(op, E_c, dE, a, dev(v)))
    phi, th = math.acos(lam_t), np.arccos((E - E_c) / dE)

    def Dk(u):
        u = np.abs(np.remainder(u + np.pi, 2 * np.pi) - np.pi)
        out = np.full_like(u, 2 * K + 1.0)
        nz = u > 1e-12
        out[nz] = np.sin((K + 0.5) * u[nz]) / np.sin(u[nz] / 2)
        return out
    P = (Dk(th - phi) + Dk(th + phi)) / (Dk(np.array([0.0]))[0] + Dk(np.array([2 * phi]))[0])
    assert np.max(np.abs(got - P * v)) <= 1e-11 * np.max(np.abs(v))


# ------------------------------------------------------------ bounds/solve ----

@pytest.mark.parametrize("case", [OPS[0], OPS[4], OPS[7], OPS[3]],
                         ids=lambda c: "-".join(map(str, c)))
def test_bounds_match_oracle(pk, ctx, case):
    say(f"bounds {case}")
    op, H = make_op(pk, ctx, *case)
    lo, hi = pk.bounds(op, dev(wl.start_vector(op.D, 0)))
    rlo, rhi = lanczos.spectral_extremes(H)
    w = rhi - rlo
    assert abs(lo - rlo) <= 1e-8 * w and abs(hi - rhi) <= 1e-8 * w


def _check_solve(pk, op, H, n_ev, lam, **kw):
    x0 = dev(wl.start_vector(op.D, 0))
    evals, evecs, res, rep, status = pk.solve(op, x0, n_ev, lam, "absolute", **kw)
    E = host(evals)
    U = host(evecs)
    R = host(res)
    Er, Ur = dense.nearest_eigenpairs(H, lam, n_ev)
    rel = np.abs(E - Er) / np.maximum(np.abs(Er), 1.0)
    ov = np.abs(np.sum(U * Ur, axis=0))
    true_res = np.linalg.norm(H @ U - U * E, axis=0)
    say(f"   K={rep['K']} iters={rep['iters']} max rel dE={rel.max():.2e} "
        f"max res={R.max():.2e} min ov={ov.min():.12f}")
    assert status == "OK"
    assert rel.max() <= 1e-10
    assert R.max() <= 1e-8 and true_res.max() <= 1e-8
    assert np.max(np.abs(true_res - R)) <= 1e-10
    assert ov.min() >= 1 - 1e-8
    return rep


@pytest.mark.parametrize("case,n_ev", [(OPS[0], 20), (OPS[4], 20), (OPS[7], 20),
                                       (("xxz", 14, 7, 3.0, 3, True), 50),
                                       (OPS[1], 15), (OPS[2], 10)],
                         ids=lambda c: "-".join(map(str, c)) if isinstance(c, tuple) else str(c))
def test_solve_matches_dense(pk, ctx, case, n_ev):
    say(f"solve {case} n_ev={n_ev}")
    op, H = make_op(pk, ctx, *case)
    E_min, E_max = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("normalized", 0.5, E_min, E_max)
    _check_solve(pk, op, H, n_ev, lam)


def test_solve_csr_storage_and_off_center(pk, ctx):
    say("solve csr off-center")
    op, H = make_op(pk, ctx, "xxz", 12, 6, 3.0, 4, True)
    op.materialize_csr().set_storage(pk.CSR)
    E_min, E_max = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("rescaled", 0.3, E_min, E_max)
    _check_solve(pk, op, H, 15, lam)


def test_solve_fp32_bulk_filter(pk, ctx):
    say("solve fp32 bulk")
    op, H = make_op(pk, ctx, *OPS[0])
    E_min, E_max = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("normalized", 0.5, E_min, E_max)
    _check_solve(pk, op, H, 20, lam, precision=pk.FP32)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_solve_graph_replay_matches_direct_launches(pk, ctx, prec):
    """The filter recurrence replayed as one HIP graph per Lanczos iteration
    (graph=1: a replay every iteration, with the eager reorthogonalization
    and checks in between) gives the eigenpairs of direct launches (graph=2)
    and of the dense oracle."""
    say(f"solve graph vs direct {prec}")
    op, H = make_op(pk, ctx, *OPS[0])
    E_min, E_max = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("normalized", 0.5, E_min, E_max)
    p = pk.FP64 if prec == "fp64" else pk.FP32
    rep_g = _check_solve(pk, op, H, 20, lam, precision=p, graph=1)
    rep_d = _check_solve(pk, op, H, 20, lam, precision=p, graph=2)
    assert rep_g["iters"] == rep_d["iters"] or prec == "fp32"


def test_graph_solve_tunes_step_kernel_before_capture(pk, ctx):
    """A solve whose first FP32 filter is recorded into a graph (graph=1)
    still picks the FP32 step kernel by timing: the tuner runs on the
    library stream before the capture (it cannot time launches inside one),
    so the captured recurrence uses the tuned variant, not the default."""
    say("graph solve tunes before capture")
    op, H = make_op(pk, ctx, *OPS[0])
    assert op.set_kernel(pk.FP32, -2) == -1  # a fresh operator is not tuned
    E_min, E_max = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("normalized", 0.5, E_min, E_max)
    _check_solve(pk, op, H, 20, lam, precision=pk.FP32, graph=1, refine_max=-1)
    assert op.set_kernel(pk.FP32, -2) >= 0


def test_fp32_refinement_fallback_to_fp64(pk, ctx):
    """With no refinement sweeps allowed, an FP32-bulk solve hands over to the
    FP64 filter and still returns the dense oracle's pairs."""
    say("fp32 fallback forced")
    op, H = make_op(pk, ctx, *OPS[0])
    E_min, E_max = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("normalized", 0.5, E_min, E_max)
    rep = _check_solve(pk, op, H, 20, lam, precision=pk.FP32, refine_max=-1)
    assert rep["fp32_fallback"] == 1


def test_fp32_stalled_refinement_case(pk, ctx):
    """XXZ L=16 W=3 seed 999, 50 pairs: a window-edge pair converges too
    slowly under the FP32 refinement; the solve must still end OK, with the
    FP64 run's eigenvalues and residuals checked with the oracle's H."""
    say("fp32 stalled case L=16")
    L = 16
    h, H, _ = xxz_case(L, L // 2, 3.0, 999)
    op = pk.Operator.xxz(ctx, L, L // 2, 1.0, 1.0, h, True)
    x0 = dev(wl.start_vector(op.D, 999))
    e32, U32, r32, rep32, st32 = pk.solve(op, x0, 50, 0.5, "normalized", precision=pk.FP32)
    e64, _, _, rep64, st64 = pk.solve(op, x0, 50, 0.5, "normalized")
    assert st32 == "OK" and st64 == "OK"
    E32, E64 = host(e32), host(e64)
    assert np.max(np.abs(E32 - E64) / np.maximum(np.abs(E64), 1.0)) <= 1e-10
    U = host(U32)
    assert np.linalg.norm(H @ U - U * E32, axis=0).max() <= 1e-8
    say(f"   fallback={rep32['fp32_fallback']} sweeps={rep32['refine_sweeps']} iters={rep32['iters']}")


# ------------------------------------------------------------ edge cases ----

@pytest.mark.parametrize("L,N", [(6, 0), (6, 6), (5, 1), (4, 2)])
def test_tiny_sectors_apply_and_step(pk, ctx, L, N):
    """Sectors of dimension 1 (no hop possible) and a few states."""
    say(f"tiny sector L={L} N={N}")
    h = wl.xxz_fields(L, 1.0, 3)
    op = pk.Operator.xxz(ctx, L, N, 1.0, 1.0, h, True)
    H, _ = models.xxz(L, N, 1.0, 1.0, h, True)
    assert op.D == H.shape[0]
    rng = np.random.default_rng(0)
    v, b1, b2 = (rng.standard_normal(op.D) for _ in range(3))
    assert np.max(np.abs(host(op.apply(dev(b1))) - H @ b1)) <= 1e-13 * max(1.0, np.max(np.abs(H @ b1)))
    tb2 = dev(b2)
    pk.clenshaw_step(op, 0.1, 3.0, 0.2, dev(v), dev(b1), tb2, pk.FP64)
    ref = 0.2 * v + 2.0 * (H @ b1 - 0.1 * b1) / 3.0 - b2
    assert np.max(np.abs(host(tb2) - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_solve_nearly_the_whole_spectrum(pk, ctx):
    """XXZ L=8 (D = 70): 50 of the 70 eigenpairs, so the Krylov space
    reaches the whole space."""
    say("solve 50 of 70 pairs")
    h = wl.xxz_fields(8, 2.0, 1)
    op = pk.Operator.xxz(ctx, 8, 4, 1.0, 1.0, h, True)
    H, _ = models.xxz(8, 4, 1.0, 1.0, h, True)
    E_min, E_max = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("normalized", 0.5, E_min, E_max)
    _check_solve(pk, op, H, 50, lam)
