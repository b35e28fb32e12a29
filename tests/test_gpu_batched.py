"""Batched setup and solve: every problem of a batch gives the same results as
the same problem set up and solved alone (the batch is one block-diagonal
matrix whose reductions are taken per problem over chunks that depend only on
the problem's own size)."""

import numpy as np
import pytest
import torch

import paper_2101_12164_amd as ns
from gpu_helpers import gpu_setup, to_dev
from workloads import aniso_problem, make_problem

pytestmark = pytest.mark.gpu

K, P_OVER = 8, 4


def batch_problems():
    ps = [aniso_problem(L, th, k=K, p=P_OVER, seed=i) for i, (L, th) in enumerate([(40, 0.3), (29, 1.9), (52, 2.7)])]
    ps.append(make_problem((33, 33), (2, 2), k=K, p=P_OVER, seed=7, name="lap2d_33"))
    ps.append(make_problem((12, 12, 12), (2, 2, 2), sigma=1.0, ell=4.0, k=K, p=P_OVER, seed=9, name="logn3d_12"))
    return ps


def solve_alone(P, **kw):
    h = gpu_setup(P, **kw)
    b = torch.as_tensor(P.b(), device="cuda")
    x, out = h.solve(b, rtol=1e-8, maxit=500, hist_cap=600)
    info = dict(h.setup_info)
    h.close()
    return x, out, info


def solve_batched(Ps, **kw):
    devs = [to_dev(P) for P in Ps]
    probs = [(d["row_ptr"], d["col"], d["val"], d["part"]) for d in devs]
    oms = [torch.as_tensor(np.ascontiguousarray(P.omega()), device="cuda") for P in Ps]
    h, infos = ns.nystrom_schur_setup_batched(probs, k=K, p=P_OVER, omegas=oms, tol_inner=0.1, **kw)
    try:
        bs = [torch.as_tensor(P.b(), device="cuda") for P in Ps]
        xs, outs = ns.nystrom_schur_pcg_solve_batched(h, bs, rtol=1e-8, maxit=500, hist_cap=600)
        sizes = ns.nystrom_schur_get_sizes(h)
    finally:
        ns.nystrom_schur_destroy(h)
    return xs, outs, infos, sizes


MODES = {
    "m2_fp64": dict(),
    "adef2": dict(apply_mode=ns.NS_APPLY_ADEF2),
    "fp32_inner": dict(prec_inner=ns.NS_FP32),
    "triangular": dict(schur_mode=ns.NS_SCHUR_TRIANGULAR),
}


@pytest.mark.parametrize("mode", list(MODES))
def test_batched_equals_alone(mode):
    Ps = batch_problems()
    kw = MODES[mode]
    alone = [solve_alone(P, **kw) for P in Ps]
    xs, outs, infos, sizes = solve_batched(Ps, **kw)
    assert sizes["nprob"] == len(Ps)
    assert sizes["n"] == sum(P.n for P in Ps)
    assert sizes["n_gamma"] == sum(P.n_gamma for P in Ps)
    for q, P in enumerate(Ps):
        x1, o1, i1 = alone[q]
        print(P.name, i1["it_inner"], infos[q]["it_inner"], o1["it_pcg"], outs[q]["it_pcg"], flush=True)
        for key in ("n", "n_gamma", "n_interior", "n_junction", "n_sub", "n_level2_blocks", "k_eff", "it_inner",
                    "inner_converged"):
            assert infos[q][key] == i1[key], (P.name, key)
        assert infos[q]["inner_relres"] == pytest.approx(i1["inner_relres"], rel=1e-12, abs=0)
        assert outs[q]["it_pcg"] == o1["it_pcg"]
        assert outs[q]["converged"] == 1
        np.testing.assert_allclose(outs[q]["res_hist"], o1["res_hist"], rtol=1e-10, atol=0)
        d = (xs[q] - x1).norm().item() / x1.norm().item()
        assert d <= 1e-13, (P.name, d)
        assert outs[q]["relres_true"] <= 1e-8


def test_batched_single_problem_is_bitwise_alone():
    P = batch_problems()[0]
    x1, o1, i1 = solve_alone(P)
    xs, outs, infos, _ = solve_batched([P])
    assert torch.equal(xs[0], x1)
    assert outs[0]["it_pcg"] == o1["it_pcg"]
    assert infos[0]["it_inner"] == i1["it_inner"]


def test_batched_rejects_bad_problem():
    Ps = batch_problems()[:2]
    devs = [to_dev(P) for P in Ps]
    bad_col = devs[1]["col"].clone()
    bad_col[5] = Ps[1].n + 3  # column outside the problem
    probs = [(devs[0]["row_ptr"], devs[0]["col"], devs[0]["val"], devs[0]["part"]),
             (devs[1]["row_ptr"], bad_col, devs[1]["val"], devs[1]["part"])]
    oms = [torch.as_tensor(np.ascontiguousarray(P.omega()), device="cuda") for P in Ps]
    with pytest.raises(ns.NsError) as e:
        ns.nystrom_schur_setup_batched(probs, k=K, p=P_OVER, omegas=oms)
    assert e.value.status == ns.NS_ERR_INVALID_ARG


@pytest.mark.parametrize("graph", [1, 3])
def test_graph_pcg_equals_plain_launches(graph):
    """PCG iterations replayed from a HIP graph give the same iterates as plain launches; two solves in a
    row on one handle (eager work and synchronisations between the replays)."""
    P = batch_problems()[2]
    rng = np.random.default_rng(5)
    b1 = torch.as_tensor(P.b(), device="cuda")
    b2 = torch.as_tensor(rng.standard_normal(P.n), device="cuda")
    res = {}
    for mode in (-1, graph):
        h = gpu_setup(P, pcg_graph_iters=mode)
        out = []
        for b in (b1, b2):
            x, o = h.solve(b, rtol=1e-8, maxit=500, hist_cap=600)
            out.append((x.clone(), o))
        h.close()
        res[mode] = out
    for (xe, oe), (xg, og) in zip(res[-1], res[graph]):
        assert og["it_pcg"] == oe["it_pcg"]
        assert og["res_hist"] == oe["res_hist"]
        assert torch.equal(xg, xe)


def test_graph_pcg_batched_equals_plain_launches():
    Ps = batch_problems()
    xe, oe, _, _ = solve_batched(Ps, pcg_graph_iters=-1)
    xg, og, _, _ = solve_batched(Ps, pcg_graph_iters=4)
    for q in range(len(Ps)):
        assert og[q]["it_pcg"] == oe[q]["it_pcg"]
        assert og[q]["res_hist"] == oe[q]["res_hist"]
        assert torch.equal(xg[q], xe[q])
