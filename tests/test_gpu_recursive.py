"""GPU: the recursive construction (NS_LEVEL2_NYSTROM) against the FP64 oracle's RecursiveGamma.

A_Gamma, split by the level-2 labels into interface blocks (its interior) and junction nodes (its interface),
is preconditioned by its block LDL^T solve with the junction Schur complement's inverse replaced by the
Nystrom-Schur preconditioner M_J of that level; every level-1 solve with A_Gamma uses it.  Both sides get the
same level-2 sketch.  Checks: the approximate A_Gamma^{-1} element by element, M r, the counts of both levels
(within one), k_eff of both levels, the 1e-8 true residual; with a full-rank level-2 sketch and a tight
level-2 tolerance the recursive solve is the exact A_Gamma^{-1}; graph-replayed and plain block CG agree bit
for bit; unsupported combinations are rejected."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2101_12164_amd as ns  # noqa: E402
from gpu_helpers import gpu_setup, oracle, rel  # noqa: E402
from oracle import DBBD, level2_part  # noqa: E402
from workloads import config_c2, make_problem  # noqa: E402

PROBS = {
    "fd3d_14": lambda: make_problem((14, 14, 14), (2, 2, 2), sigma=0.0, ell=8.0, k=10, p=5),
    "lognormal3d_24": lambda: make_problem((24, 24, 24), (3, 3, 3), sigma=2.0, ell=6.0, k=32, p=8),
    "lognormal3d_32": lambda: make_problem((32, 32, 32), (2, 2, 2), sigma=2.0, ell=8.0, k=64, p=16),
}
LEVEL2 = {"fd3d_14": (8, 4), "lognormal3d_24": (16, 8), "lognormal3d_32": (24, 8)}


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def n_junction(P):
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    return int(np.count_nonzero(level2_part(d) == -1)), d.n_gamma


def sketch2(nJ, k2, p2, seed=7):
    return np.random.default_rng(seed).standard_normal((nJ, k2 + p2))


@pytest.mark.parametrize("name", sorted(PROBS))
def test_recursive_matches_oracle(name):
    P = PROBS[name]()
    nJ, nG = n_junction(P)
    k2, p2 = LEVEL2[name]
    om2 = sketch2(nJ, k2, p2)
    print(f"[recursive] {name}: n={P.n} n_gamma={nG} n_J={nJ} k2={k2} p2={p2}", flush=True)
    o = oracle(P, level2=dict(k=k2, p=p2, omega=om2))
    so = o.setup()
    ro = o.solve(P.b(), tol=1e-8)
    g = gpu_setup(P, level2=ns.NS_LEVEL2_NYSTROM, level2_k=k2, level2_p=p2, level2_omega=dev(om2))
    try:
        si = g.setup_info
        x, info = g.solve(dev(P.b()), rtol=1e-8, maxit=2000)
        X = np.random.default_rng(3).standard_normal((nG, 5))
        Y = ns.nystrom_schur_interface_solve(g.handle, dev(X)).cpu().numpy()
        ey = rel(Y, o.level2.solve(X))
        Mr = ns.nystrom_schur_apply(g.handle, dev(X)).cpu().numpy()
        em = rel(Mr, o.apply(X))
        print(f"[recursive] {name}: level-2 it_SI {si['level2_it_inner']} (oracle "
              f"{o.level2.setup_result.it_inner}), k_eff2 {si['level2_k_eff']}; it_SI {si['it_inner']} (oracle "
              f"{so.it_inner}), it_PCG {info['it_pcg']} (oracle {ro.it_pcg}), relres_true {info['relres_true']:.2e}; "
              f"A~^-1 X error {ey:.2e}, M X error {em:.2e}", flush=True)
        assert abs(si["level2_it_inner"] - o.level2.setup_result.it_inner) <= 1
        assert si["level2_k_eff"] == o.level2.setup_result.k_eff
        assert abs(si["it_inner"] - so.it_inner) <= 1
        assert abs(info["it_pcg"] - ro.it_pcg) <= 1
        assert info["relres_true"] <= 1e-8
        assert ey < 1e-10 and em < 1e-10
    finally:
        g.close()


def test_full_rank_level2_is_exact():
    P = PROBS["fd3d_14"]()
    nJ, nG = n_junction(P)
    om2 = sketch2(nJ, nJ, 0, seed=3)
    o = oracle(P)
    ro = o.solve(P.b(), tol=1e-8)
    g = gpu_setup(P, level2=ns.NS_LEVEL2_NYSTROM, level2_k=nJ, level2_p=0, level2_omega=dev(om2),
                  level2_tol_inner=1e-13)
    try:
        X = np.random.default_rng(1).standard_normal((nG, 3))
        Y = ns.nystrom_schur_interface_solve(g.handle, dev(X)).cpu().numpy()
        e = rel(Y, o.ops.solve_G(X))
        x, info = g.solve(dev(P.b()), rtol=1e-8, maxit=2000)
        print(f"[recursive] full-rank level 2: A~^-1 X vs exact {e:.2e}, it_PCG {info['it_pcg']} (exact oracle "
              f"{ro.it_pcg})", flush=True)
        assert e <= 1e-9
        assert abs(info["it_pcg"] - ro.it_pcg) <= 1
    finally:
        g.close()


def test_level2_rank_zero_is_first_level():
    P = PROBS["lognormal3d_24"]()
    nJ, nG = n_junction(P)
    o = oracle(P, level2=dict(k=0, p=0, omega=None))
    g = gpu_setup(P, level2=ns.NS_LEVEL2_NYSTROM, level2_k=0)
    try:
        X = np.random.default_rng(2).standard_normal((nG, 4))
        Y = ns.nystrom_schur_interface_solve(g.handle, dev(X)).cpu().numpy()
        assert rel(Y, o.level2.solve(X)) < 1e-10
        assert g.setup_info["level2_k_eff"] == 0 and g.setup_info["level2_it_inner"] == 0
    finally:
        g.close()


@pytest.mark.parametrize("combo", ["M3", "ADEF2", "outer_full", "power1"])
def test_recursive_with_other_options(combo):
    P = PROBS["lognormal3d_24"]()
    nJ, nG = n_junction(P)
    k2, p2 = LEVEL2["lognormal3d_24"]
    om2 = sketch2(nJ, k2, p2)
    okw, gkw = {}, {}
    if combo == "M3":
        nI = P.n - nG
        om = np.random.default_rng(P.seed).standard_normal((nI, P.k + P.p))
        okw = dict(variant="M3", omega=om)
        gkw = dict(variant=ns.NS_VARIANT_M3, omega=om)
    elif combo == "ADEF2":
        okw = dict(apply_mode="ADEF2")
        gkw = dict(apply_mode=ns.NS_APPLY_ADEF2)
    elif combo == "outer_full":
        gkw = dict(outer=ns.NS_OUTER_FULL)
    else:
        okw = dict(power=1)
        gkw = dict(power_iters=1)
    o = oracle(P, level2=dict(k=k2, p=p2, omega=om2), **okw)
    so = o.setup()
    if combo == "outer_full":
        from oracle import full_system_pcg

        it_ref = full_system_pcg(o, P.b(), tol=1e-8).iters
    else:
        it_ref = o.solve(P.b(), tol=1e-8).it_pcg
    g = gpu_setup(P, level2=ns.NS_LEVEL2_NYSTROM, level2_k=k2, level2_p=p2, level2_omega=dev(om2), **gkw)
    try:
        x, info = g.solve(dev(P.b()), rtol=1e-8, maxit=2000)
        si = g.setup_info
        print(f"[recursive] {combo}: it_SI {si['it_inner']} (oracle {so.it_inner}), it_PCG {info['it_pcg']} "
              f"(oracle {it_ref}), relres_true {info['relres_true']:.2e}", flush=True)
        assert abs(si["it_inner"] - so.it_inner) <= 1 + (1 if combo == "power1" else 0)
        assert abs(info["it_pcg"] - it_ref) <= 1
        assert info["relres_true"] <= 1e-8
    finally:
        g.close()


def test_graph_and_plain_block_cg_agree():
    P = PROBS["lognormal3d_24"]()
    nJ, nG = n_junction(P)
    k2, p2 = LEVEL2["lognormal3d_24"]
    om2 = dev(sketch2(nJ, k2, p2))
    R = dev(np.random.default_rng(5).standard_normal((nG, 3)))
    out = []
    for m in (-1, 0, 4):
        g = gpu_setup(P, level2=ns.NS_LEVEL2_NYSTROM, level2_k=k2, level2_p=p2, level2_omega=om2,
                      bcg_graph_iters=m, pcg_graph_iters=m)
        try:
            x, info = g.solve(dev(P.b()), rtol=1e-8, maxit=2000)
            out.append((g.setup_info["it_inner"], g.setup_info["level2_it_inner"], info["it_pcg"],
                        ns.nystrom_schur_apply(g.handle, R).cpu().numpy(), x.cpu().numpy()))
        finally:
            g.close()
    for o_ in out[1:]:
        assert o_[:3] == out[0][:3]
        assert np.array_equal(o_[3], out[0][3]) and np.array_equal(o_[4], out[0][4])


def test_recursive_rejections():
    P = PROBS["fd3d_14"]()
    nJ, nG = n_junction(P)
    om2 = dev(sketch2(nJ, 4, 2))
    for kw in (dict(prec_inner=ns.NS_FP32), dict(prec_inner=ns.NS_BF16), dict(variant=ns.NS_VARIANT_M1)):
        with pytest.raises(ns.NsError):
            gpu_setup(P, level2=ns.NS_LEVEL2_NYSTROM, level2_k=4, level2_p=2, level2_omega=om2, **kw)
    with pytest.raises(ns.NsError):  # k_2 + p_2 beyond the junction nodes
        gpu_setup(P, level2=ns.NS_LEVEL2_NYSTROM, level2_k=nJ, level2_p=1, level2_omega=dev(sketch2(nJ, nJ, 1)))
    with pytest.raises(ns.NsError):  # no sketch
        gpu_setup(P, level2=ns.NS_LEVEL2_NYSTROM, level2_k=4, level2_p=2)
    g = gpu_setup(P, level2=ns.NS_LEVEL2_NYSTROM, level2_k=4, level2_p=2, level2_omega=om2)
    try:
        with pytest.raises(ns.NsError):
            ns.nystrom_schur_apply_noalloc(g.handle, dev(np.ones((nG, 1))), dev(np.zeros((nG, 1))))
    finally:
        g.close()


def test_recursive_full_size_64cube():
    """The 64^3 lognormal system with the recursive level (1674 junction nodes, k_2 = 64, p_2 = 16) against
    the exact A_Gamma solve on the same system: both reach the 1e-8 target."""
    P = config_c2()
    nJ, nG = n_junction(P)
    om2 = dev(sketch2(nJ, 64, 16))
    res = {}
    for mode in (ns.NS_LEVEL2_EXACT, ns.NS_LEVEL2_NYSTROM):
        kw = dict(level2=mode, level2_k=64, level2_p=16, level2_omega=om2) if mode else {}
        g = gpu_setup(P, **kw)
        try:
            x, info = g.solve(dev(P.b()), rtol=1e-8, maxit=2000)
            res[mode] = (g.setup_info, info)
            print(f"[recursive] 64^3 level2={mode}: it_SI {g.setup_info['it_inner']}, level-2 it_SI "
                  f"{g.setup_info['level2_it_inner']}, it_PCG {info['it_pcg']}, relres_true {info['relres_true']:.2e}, "
                  f"setup {g.setup_info['t_total'] * 1e3:.1f} ms, solve {info['t_solve'] * 1e3:.1f} ms", flush=True)
            assert info["relres_true"] <= 1e-8
        finally:
            g.close()
    assert res[ns.NS_LEVEL2_NYSTROM][0]["level2_k_eff"] == 64
