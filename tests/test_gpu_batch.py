"""GPU parity of the multi-column path (realizations sharing the off-diagonal
pattern): each column of the batched Clenshaw step, the batched filter and
the batched solve against the CPU oracle of that column's own Hamiltonian."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense, lanczos
from oracle import filter as flt
from tests.test_gpu_parity import ctx, dev, host, pk, say, tv_case, xxz_case  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def batch_ops(pk, ctx, kind, L, B, periodic=True):
    """B realizations: XXZ with W cycling through 1, 3, 5 and seeds 0..B-1,
    or t-V with seeds 0..B-1."""
    ops, Hs = [], []
    for c in range(B):
        if kind == "xxz":
            W = (1.0, 3.0, 5.0)[c % 3]
            h, H, _ = xxz_case(L, L // 2, W, c, periodic)
            ops.append(pk.Operator.xxz(ctx, L, L // 2, 1.0, 1.0, h, periodic))
        else:
            eps, H, _ = tv_case(L, L // 2, c, periodic)
            ops.append(pk.Operator.tv(ctx, L, L // 2, 1.0, 1.0, eps, periodic))
        Hs.append(H)
    return ops, Hs


def ref_step(H, E_c, dE, a_i, v, b1, b2, final):
    f = 0.5 if final else 1.0
    return a_i * v + f * 2.0 * (H @ b1 - E_c * b1) / dE - b2


STEP_CASES = [("xxz", 12, 3, True), ("xxz", 14, 5, True), ("xxz", 16, 2, True),
              ("tv", 12, 4, True), ("xxz", 10, 20, True), ("xxz", 18, 3, True),
              ("xxz", 13, 3, False), ("tv", 11, 2, False)]


@pytest.mark.parametrize("case", STEP_CASES, ids=lambda c: "-".join(map(str, c)))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("final", [False, True])
def test_clenshaw_step_batch_matches_oracle(pk, ctx, case, prec, final):
    kind, L, B, periodic = case
    say(f"batch step {case} {prec} final={final}")
    ops, Hs = batch_ops(pk, ctx, kind, L, B, periodic)
    D = ops[0].D
    rng = np.random.default_rng(21)
    V, B1, B2 = (rng.standard_normal((B, D)) for _ in range(3))
    E_c = rng.uniform(-0.5, 0.5, B)
    dE = rng.uniform(6.0, 12.0, B)
    a_i = rng.uniform(-0.1, 0.1, B)
    dt = torch.float64 if prec == "fp64" else torch.float32
    tb2 = dev(B2, dt)
    pk.clenshaw_step_batch(ops, E_c, dE, a_i, dev(V, dt), dev(B1, dt), tb2,
                           pk.FP64 if prec == "fp64" else pk.FP32, final)
    got = host(tb2).astype(np.float64)
    tol = 1e-14 if prec == "fp64" else 2e-6
    for c in range(B):
        ref = ref_step(Hs[c], E_c[c], dE[c], a_i[c], V[c], B1[c], B2[c], final)
        err = np.max(np.abs(got[c] - ref)) / np.max(np.abs(ref))
        assert err <= tol, (c, err)


def filter_tol(K, prec):
    eps = 2.2e-16 if prec == "fp64" else 1.2e-7
    return 8 * (K + 1) * eps


@pytest.mark.parametrize("case,Ks", [(("xxz", 12, 3), [300, 281, 150]),
                                     (("xxz", 14, 4), [700, 0, 1, 2]),
                                     (("xxz", 14, 1), [573]),
                                     (("tv", 12, 2), [400, 400]),
                                     (("xxz", 10, 18), list(range(40, 58))),
                                     (("xxz", 12, 21), [90 + 3 * c for c in range(21)]),
                                     (("xxz", 16, 32), [60 - (c % 7) for c in range(32)])],
                         ids=lambda c: "-".join(map(str, c[:3])) if isinstance(c[0], str) else "K")
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", [-1, 0, 1, 2, 3, 5, 6, 7])
def test_filter_apply_batch_matches_oracle(pk, ctx, case, Ks, prec, variant):
    """Every column of the batched filter against the oracle's filter of its
    own Hamiltonian, element by element, with the tuned multi-column kernel
    and with each variant forced (column-major blocks with 16 or 8 columns
    per launch; interleaved blocks, including a last group narrower than a
    16-byte access for odd batch widths; the LDS-resident whole filter with
    each column's own order, K = 0 included; the row-group kernel, with
    lanes past the last column for widths that do not fill a power of two of
    16-byte groups, up to 32 columns)."""
    kind, L, B = case
    say(f"batch filter {case} K={Ks[:4]} {prec} variant {variant}")
    ops, Hs = batch_ops(pk, ctx, kind, L, B)
    p = pk.FP64 if prec == "fp64" else pk.FP32
    if variant == 5 and L > 14:
        # the LDS-resident filter where two vectors and the tables fit the
        # LDS (FP64 to L = 14; FP32 beyond only for some chains), else refused
        try:
            ops[0].set_batch_kernel(B, p, variant)
        except pk.PolfedError as e:
            assert "LDS" in str(e)
            return
    assert ops[0].set_batch_kernel(B, p, variant) == variant
    D = ops[0].D
    E_c, dE, coefs, refs = [], [], [], []
    V = np.stack([wl.start_vector(D, 30 + c) for c in range(B)])
    for c in range(B):
        lo, hi = lanczos.spectral_extremes(Hs[c])
        ec, de = flt.rescale(*lanczos.padded_bounds(lo, hi, 1e-3))
        a = flt.coefficients(-0.2 + 0.1 * (c % 5), Ks[c])
        E_c.append(ec)
        dE.append(de)
        coefs.append(a)
        refs.append(flt.apply_filter(Hs[c], ec, de, a, V[c]))
    dt = torch.float64 if prec == "fp64" else torch.float32
    w = pk.filter_apply_batch(ops, E_c, dE, coefs, dev(V, dt),
                              pk.FP64 if prec == "fp64" else pk.FP32)
    got = host(w).astype(np.float64)
    for c in range(B):
        err = np.linalg.norm(got[c] - refs[c]) / np.linalg.norm(refs[c])
        err_el = np.max(np.abs(got[c] - refs[c])) / np.max(np.abs(refs[c]))
        assert err <= filter_tol(max(Ks), prec), (c, Ks[c], err)
        assert err_el <= filter_tol(max(Ks), prec), (c, Ks[c], err_el)


def test_batch_rejects_mixed_patterns(pk, ctx):
    say("batch mixed patterns")
    a, _ = batch_ops(pk, ctx, "xxz", 12, 1)
    b, _ = batch_ops(pk, ctx, "xxz", 14, 1)
    c, _ = batch_ops(pk, ctx, "tv", 12, 1)
    v = torch.zeros((2, a[0].D), dtype=torch.float64, device="cuda:0")
    for pair in ([a[0], b[0]], [a[0], c[0]]):
        with pytest.raises(pk.PolfedError) as e:
            pk.filter_apply_batch(pair, [0, 0], [1, 1], [[1.0], [1.0]], v)
        assert "pattern" in str(e.value)


def _check_pairs(H, lam, n_ev, evals, evecs, res):
    E, U, R = host(evals), host(evecs), host(res)
    Er, Ur = dense.nearest_eigenpairs(H, lam, n_ev)
    rel = np.abs(E - Er) / np.maximum(np.abs(Er), 1.0)
    ov = np.abs(np.sum(U * Ur, axis=0))
    true_res = np.linalg.norm(H @ U - U * E, axis=0)
    assert rel.max() <= 1e-10
    assert R.max() <= 1e-8 and true_res.max() <= 1e-8
    assert ov.min() >= 1 - 1e-8
    return rel.max(), R.max()


@pytest.mark.parametrize("kind,L,B,n_ev", [("xxz", 12, 3, 20), ("xxz", 14, 4, 50),
                                           ("tv", 12, 3, 20)])
def test_solve_batch_matches_dense(pk, ctx, kind, L, B, n_ev):
    say(f"solve_batch {kind} L={L} B={B} n_ev={n_ev}")
    ops, Hs = batch_ops(pk, ctx, kind, L, B)
    x0s = [dev(wl.start_vector(o.D, c)) for c, o in enumerate(ops)]
    out, status = pk.solve_batch(ops, x0s, n_ev, 0.5, "normalized")
    assert status == "OK"
    for c, (ev, U, R, rep) in enumerate(out):
        rel, res = _check_pairs(Hs[c], rep["lambda"], n_ev, ev, U, R)
        say(f"   col {c}: K={rep['K']} iters={rep['iters']} rel={rel:.1e} res={res:.1e}")


def test_solve_batch_equals_single_solves(pk, ctx):
    """Each realization gives the same eigenpairs in the batch as alone."""
    say("solve_batch vs single")
    ops, Hs = batch_ops(pk, ctx, "xxz", 12, 3)
    x0s = [dev(wl.start_vector(o.D, c)) for c, o in enumerate(ops)]
    out, _ = pk.solve_batch(ops, x0s, 20, 0.5, "normalized")
    for c, op in enumerate(ops):
        ev1, U1, _, rep1, st = pk.solve(op, x0s[c], 20, 0.5, "normalized")
        assert st == "OK"
        evb, Ub = host(out[c][0]), host(out[c][1])
        assert abs(rep1["lambda"] - out[c][3]["lambda"]) <= 1e-12 * max(1.0, abs(rep1["lambda"]))
        assert np.max(np.abs(host(ev1) - evb) / np.maximum(np.abs(evb), 1.0)) <= 1e-10
        ov = np.abs(np.sum(host(U1) * Ub, axis=0))
        assert ov.min() >= 1 - 1e-8


def test_solve_batch_graph_replay(pk, ctx):
    """Batched filter replayed as a HIP graph every iteration."""
    say("solve_batch graph replay")
    ops, Hs = batch_ops(pk, ctx, "xxz", 12, 3)
    x0s = [dev(wl.start_vector(o.D, c)) for c, o in enumerate(ops)]
    out, status = pk.solve_batch(ops, x0s, 20, 0.5, "normalized", graph=1)
    assert status == "OK"
    for c, (ev, U, R, rep) in enumerate(out):
        _check_pairs(Hs[c], rep["lambda"], 20, ev, U, R)


@pytest.mark.parametrize("kind,L,B,n_ev", [("xxz", 12, 3, 20), ("xxz", 14, 4, 50),
                                           ("tv", 12, 3, 20)])
def test_solve_batch_fp32_bulk_matches_dense(pk, ctx, kind, L, B, n_ev):
    """FP32 recurrence for the whole batch, FP64 reorthogonalization,
    Rayleigh-Ritz and refinement: every column meets the FP64 bar against
    the dense FP64 oracle, and its per-eigenpair error is reported."""
    say(f"solve_batch FP32 bulk {kind} L={L} B={B} n_ev={n_ev}")
    ops, Hs = batch_ops(pk, ctx, kind, L, B)
    x0s = [dev(wl.start_vector(o.D, c)) for c, o in enumerate(ops)]
    out, status = pk.solve_batch(ops, x0s, n_ev, 0.5, "normalized", precision=pk.FP32)
    assert status == "OK"
    for c, (ev, U, R, rep) in enumerate(out):
        assert rep["precision"] == pk.FP32
        rel, res = _check_pairs(Hs[c], rep["lambda"], n_ev, ev, U, R)
        say(f"   col {c}: K={rep['K']} iters={rep['iters']} sweeps={rep['refine_sweeps']} "
            f"fallback={rep['fp32_fallback']} max rel dE={rel:.1e} max res={res:.1e}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_kernel_is_tuned_and_kept(pk, ctx, prec):
    """The first batched filter of a pattern picks the multi-column kernel by
    timing and keeps it for that batch width; the result meets the bar."""
    say(f"batch kernel tuning {prec}")
    ops, Hs = batch_ops(pk, ctx, "xxz", 16, 6)
    p = pk.FP64 if prec == "fp64" else pk.FP32
    assert ops[0].set_batch_kernel(6, p, -2) == -1
    D = ops[0].D
    V = np.stack([wl.start_vector(D, 70 + c) for c in range(6)])
    dt = torch.float64 if prec == "fp64" else torch.float32
    coefs = [flt.coefficients(0.1, 50) for _ in range(6)]
    w = pk.filter_apply_batch(ops, [0.0] * 6, [30.0] * 6, coefs, dev(V, dt), p)
    chosen = ops[0].set_batch_kernel(6, p, -2)
    say(f"   chosen variant {chosen}")
    assert chosen in (0, 1, 2, 3, 5, 6, 7)
    got = host(w).astype(np.float64)
    for c in range(6):
        ref = flt.apply_filter(Hs[c], 0.0, 30.0, coefs[c], V[c])
        assert np.max(np.abs(got[c] - ref)) <= filter_tol(50, prec) * np.max(np.abs(ref))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_per_column_tile_kernels_long_chain(pk, ctx, prec):
    """Variant 4 (each column stepped by its own operator's tuned
    single-column kernel, the staged-tile kernels of long chains) on three
    L = 22 realizations: every column element by element against the
    oracle's filter of its own Hamiltonian (D = 705,432, K = 20); the same
    variant is refused below L = 22."""
    say(f"batch variant 4, L=22, {prec}")
    ops, Hs = batch_ops(pk, ctx, "xxz", 22, 3)
    p = pk.FP64 if prec == "fp64" else pk.FP32
    assert ops[0].set_batch_kernel(3, p, 4) == 4
    D = ops[0].D
    V = np.stack([wl.start_vector(D, 90 + c) for c in range(3)])
    coefs = [flt.coefficients(0.05 * c, 20) for c in range(3)]
    E_c, dE = [0.1, -0.2, 0.0], [40.0, 45.0, 50.0]
    dt = torch.float64 if prec == "fp64" else torch.float32
    w = pk.filter_apply_batch(ops, E_c, dE, coefs, dev(V, dt), p)
    got = host(w).astype(np.float64)
    for c in range(3):
        ref = flt.apply_filter(Hs[c], E_c[c], dE[c], coefs[c], V[c])
        assert np.max(np.abs(got[c] - ref)) <= filter_tol(20, prec) * np.max(np.abs(ref))
    small, _ = batch_ops(pk, ctx, "xxz", 12, 2)
    with pytest.raises(pk.PolfedError):
        small[0].set_batch_kernel(2, p, 4)
