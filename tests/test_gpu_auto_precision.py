"""GPU tests of the automatic filter precision (FP32 bulk where its step is
clearly faster, else FP64): whichever precision the timing picks, solves,
batches and served requests meet the FP64 bar against the dense oracle, the
choice is kept per operator and reported, and the step calls, which take an
explicit precision, reject it."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense, lanczos, polfed
from tests.test_gpu_batch import batch_ops
from tests.test_gpu_parity import OPS, ctx, dev, host, make_op, pk, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _check(H, lam, n_ev, ev, U, R):
    E, Uh, Rh = host(ev), host(U), host(R)
    Er, Ur = dense.nearest_eigenpairs(H, lam, n_ev)
    rel = np.abs(E - Er) / np.maximum(np.abs(Er), 1.0)
    assert rel.max() <= 1e-10
    assert Rh.max() <= 1e-8
    assert np.linalg.norm(H @ Uh - Uh * E, axis=0).max() <= 1e-8
    assert np.abs(np.sum(Uh * Ur, axis=0)).min() >= 1 - 1e-8
    return rel.max()


@pytest.mark.parametrize("case", [OPS[0], OPS[4], OPS[7]],
                         ids=lambda c: "-".join(map(str, c)))
def test_auto_solve_matches_dense_and_keeps_its_choice(pk, ctx, case):
    say(f"auto precision solve {case}")
    op, H = make_op(pk, ctx, *case)
    E_min, E_max = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("normalized", 0.5, E_min, E_max)
    x0 = dev(wl.start_vector(op.D, 0))
    ev, U, R, rep, st = pk.solve(op, x0, 20, lam, "absolute", precision=pk.AUTO)
    assert st == "OK"
    assert rep["precision"] in (pk.FP64, pk.FP32)
    rel = _check(H, lam, 20, ev, U, R)
    say(f"   picked {'FP32 bulk' if rep['precision'] == pk.FP32 else 'FP64'}: "
        f"iters={rep['iters']} rel={rel:.1e}")
    _, _, _, rep2, st2 = pk.solve(op, x0, 20, lam, "absolute", precision=pk.AUTO)
    assert st2 == "OK" and rep2["precision"] == rep["precision"]
    # an explicit precision is reported as given
    for prec in (pk.FP64, pk.FP32):
        _, _, _, rep3, st3 = pk.solve(op, x0, 20, lam, "absolute", precision=prec)
        assert st3 == "OK" and rep3["precision"] == prec


def test_auto_batch_and_served_requests(pk, ctx):
    say("auto precision batch and serve")
    n_ev = 20
    ops, Hs = batch_ops(pk, ctx, "xxz", 12, 3)
    x0s = [dev(wl.start_vector(o.D, c)) for c, o in enumerate(ops)]
    out, status = pk.solve_batch(ops, x0s, n_ev, 0.5, "normalized", precision=pk.AUTO)
    assert status == "OK"
    assert len({rep["precision"] for (_, _, _, rep) in out}) == 1
    for c, (ev, U, R, rep) in enumerate(out):
        _check(Hs[c], rep["lambda"], n_ev, ev, U, R)
    with pk.Server(ctx, 8 << 30, max_cols=4) as srv:
        reqs = [srv.submit(op, x0s[i], n_ev, 0.5, "normalized", precision=pk.AUTO)
                for i, op in enumerate(ops)]
        results = [r.wait() for r in reqs]
    for i, (ev, U, R, rep, st) in enumerate(results):
        assert st == "OK" and rep["precision"] in (pk.FP64, pk.FP32)
        _check(Hs[i], rep["lambda"], n_ev, ev, U, R)
    # the batch timed ops[0]; its served request keeps that choice
    assert results[0][3]["precision"] == out[0][3]["precision"]


def test_step_calls_reject_auto(pk, ctx):
    say("auto precision rejected by step calls")
    op, _ = make_op(pk, ctx, *OPS[0])
    v, b1, b2 = (dev(np.ones(op.D)) for _ in range(3))
    with pytest.raises(pk.PolfedError):
        pk.clenshaw_step(op, 0.0, 10.0, 0.0, v, b1, b2, pk.AUTO)
    with pytest.raises(pk.PolfedError):
        pk.profile_step(op, pk.AUTO, 5)
