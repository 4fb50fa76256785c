"""The allocation-free filter application (polfed_filter_apply_noalloc,
recurrence buffers in the library's static device scratch) against the
allocating polfed_filter_apply: the same w = P(H~) v, element by element,
on consecutive calls with shrinking inputs (the scratch keeps the previous
call's contents), at the metric's chain size, in both precisions; and its
refusals (a size beyond the scratch, an operator whose step kernel has not
been chosen yet)."""
import numpy as np
import pytest

import workloads as wl
from oracle import filter as flt
from tests.test_gpu_parity import ctx, dev, host, pk, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _coefs(K, lam_t=0.1):
    return np.asarray(flt.coefficients(lam_t, K))


def _pair(pk, op, L, prec, K, seed):
    dt = torch.float64 if prec == pk.FP64 else torch.float32
    v = dev(np.random.default_rng(seed).standard_normal(op.D), dt)
    a = _coefs(K)
    E_c, dE = 0.2, 3.0 * L + 10.0
    ref = pk.filter_apply(op, E_c, dE, a, v, prec)  # allocating path (also tunes)
    w = torch.full_like(v, float("nan"))
    pk.filter_apply_noalloc(op, E_c, dE, a, v, w, prec)
    torch.cuda.synchronize()
    got, want = host(w).astype(np.float64), host(ref).astype(np.float64)
    assert np.all(np.isfinite(got))
    tol = 0.0  # same kernels, same order: the results are identical
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want))
    return got


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_filter_matches_allocating_filter(pk, ctx, prec):
    p = pk.FP64 if prec == "fp64" else pk.FP32
    say(f"noalloc filter {prec}: L=16, then L=14, then L=24")
    for L, K, seed in ((16, 300, 1), (14, 150, 2), (24, 12, 3)):
        op = pk.Operator.xxz(ctx, L, L // 2, 1.0, 1.0, wl.xxz_fields(L, 3.0, seed), True)
        if L == 16:
            # a fresh operator: its step kernel is chosen by timing, which
            # allocates, so the allocation-free call refuses it
            v = dev(np.ones(op.D), torch.float64 if p == pk.FP64 else torch.float32)
            with pytest.raises(pk.PolfedError) as e:
                pk.filter_apply_noalloc(op, 0.0, 20.0, _coefs(10), v, torch.empty_like(v), p)
            assert "not chosen" in str(e.value)
        _pair(pk, op, L, p, K, seed)
        say(f"   L={L} D={op.D} K={K}: identical")


def test_noalloc_filter_quantum_sun_and_size_limit(pk, ctx):
    say("noalloc filter: quantum sun; QREM L=22 beyond the FP64 scratch, within FP32")
    q = wl.qsun_draws(3, 9, 0)
    op = pk.Operator.qsun(ctx, 3, 9, q["A"], 1.0, 1.0, 0.75, q["u"], q["n_of_j"], q["h"])
    _pair(pk, op, 12, pk.FP64, 200, 4)
    qr = pk.Operator.qrem(ctx, 22, wl.qrem_energies(22, 0), 1.0)
    v = dev(np.random.default_rng(5).standard_normal(qr.D))
    with pytest.raises(pk.PolfedError) as e:
        pk.filter_apply_noalloc(qr, 0.0, 30.0, _coefs(10), v, torch.empty_like(v), pk.FP64)
    assert "scratch" in str(e.value)
    _pair(pk, qr, 22, pk.FP32, 10, 6)
