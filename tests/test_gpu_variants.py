"""GPU: the method variants M_1 and M_3 with their adapted-deflation forms, power iterations of the sketch and the
full-system outer iteration, through the C ABI, against the FP64 oracle.

Tolerances as in the parity tests: it_SI within +-1 per inner solve, it_PCG within +-1, the relative residual
1e-8 reached, M r within 1e-7 of the oracle when both took the same inner iterations (the low-rank terms then
differ by the rounding of the inner solves only)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2101_12164_amd as ns  # noqa: E402
from gpu_helpers import gpu_setup, oracle, rel  # noqa: E402
from oracle import full_system_pcg  # noqa: E402
from workloads import config_c1, make_problem  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


PROBS = {
    "c1": lambda: config_c1(),
    "fd2d_40x36": lambda: make_problem((40, 36), (3, 2), sigma=1.5, ell=4.0, k=6, p=4),
    "fd3d_16": lambda: make_problem((16, 16, 16), (2, 2, 2), sigma=2.0, ell=4.0, k=12, p=6),
}
VARIANTS = {"M1": ns.NS_VARIANT_M1, "M2": ns.NS_VARIANT_M2, "M3": ns.NS_VARIANT_M3}
MODES = {"M2": ns.NS_APPLY_M2, "ADEF2": ns.NS_APPLY_ADEF2}


def interior_sketch(P):
    nI = int(np.count_nonzero(P.part >= 0))
    return np.random.default_rng(100 + P.seed).standard_normal((nI, P.k + P.p))


CASES = [(p, v, m, q) for p in sorted(PROBS) for v in ("M1", "M3") for m in ("M2", "ADEF2") for q in (0,)]
CASES += [(p, "M2", m, 1) for p in sorted(PROBS) for m in ("M2", "ADEF2")]
CASES += [("fd3d_16", "M1", "M2", 1), ("fd3d_16", "M3", "M2", 1)]


@pytest.mark.parametrize("pname,variant,mode,q", CASES, ids=[f"{a}-{b}-{c}-q{d}" for a, b, c, d in CASES])
def test_variant_matches_oracle(pname, variant, mode, q):
    P = PROBS[pname]()
    om = interior_sketch(P) if variant == "M3" else P.omega()
    print(f"[variants] {pname} variant={variant} mode={mode} q={q}", flush=True)
    o = oracle(P, variant=variant, apply_mode=mode, power=q, omega=om)
    r = o.solve(P.b(), tol=P.tol_outer)
    g = gpu_setup(P, omega=om, variant=VARIANTS[variant], apply_mode=MODES[mode], power_iters=q)
    try:
        si = g.setup_info
        assert abs(si["it_inner"] - o.setup_result.it_inner) <= q + 1, (si["it_inner"], o.setup_result.it_inner)
        assert si["k_eff"] == o.setup_result.k_eff
        if si["it_inner"] == o.setup_result.it_inner:
            R = np.random.default_rng(5).standard_normal((o.dbbd.n_gamma, 3))
            Z = ns.nystrom_schur_apply(g.handle, dev(R)).cpu().numpy()
            assert rel(Z, o.apply(R)) < 1e-7
        x, info = g.solve(dev(P.b()), rtol=P.tol_outer, maxit=500)
        assert info["converged"] == 1
        assert abs(info["it_pcg"] - r.it_pcg) <= 1, (info["it_pcg"], r.it_pcg)
        assert info["relres_true"] <= 1e-8
        assert rel(x.cpu().numpy(), r.x) < 1e-6
    finally:
        g.close()


@pytest.mark.parametrize("variant", ["M1", "M3"])
def test_variant_fp32_inner(variant):
    """FP32 inner block CG for the variants: counts within +-1 of the FP64 oracle, 1e-8 still reached."""
    P = PROBS["fd3d_16"]()
    om = interior_sketch(P) if variant == "M3" else P.omega()
    o = oracle(P, variant=variant, omega=om)
    r = o.solve(P.b(), tol=1e-8)
    g = gpu_setup(P, omega=om, variant=VARIANTS[variant], prec_inner=ns.NS_FP32)
    try:
        x, info = g.solve(dev(P.b()), rtol=1e-8)
        assert abs(g.setup_info["it_inner"] - o.setup_result.it_inner) <= 1
        assert abs(info["it_pcg"] - r.it_pcg) <= 1
        assert info["relres_true"] <= 1e-8
    finally:
        g.close()


def test_m1_full_rank_is_exact_inverse():
    """Nystrom of the whole interface with an exact inner solve: M_1 = S^{-1}, one PCG iteration."""
    P = make_problem((12, 12), (2, 2), sigma=1.0, ell=3.0, k=4, p=3)
    ng = P.n_gamma
    om = np.random.default_rng(5).standard_normal((ng, ng))
    g = gpu_setup(P, omega=om, k=ng, p=0, tol_inner=1e-13, eig_thresh_rel=1e-14, variant=ns.NS_VARIANT_M1)
    try:
        x, info = g.solve(dev(P.b()), rtol=1e-8)
        assert info["it_pcg"] == 1 and info["relres_true"] <= 1e-8
    finally:
        g.close()


@pytest.mark.parametrize("pname", sorted(PROBS))
def test_full_system_outer_matches_oracle(pname):
    """PCG on A x = b with the block LDL^T preconditioner (S~^{-1} = M_2): iterations within +-1 of the oracle's
    full-system PCG, true relative residual 1e-8."""
    P = PROBS[pname]()
    o = oracle(P)
    o.setup()
    ref = full_system_pcg(o, P.b(), tol=1e-8, maxit=1000)
    g = gpu_setup(P, outer=ns.NS_OUTER_FULL)
    try:
        x, info = g.solve(dev(P.b()), rtol=1e-8, maxit=1000)
        assert info["converged"] == 1
        assert abs(info["it_pcg"] - ref.iters) <= 1, (info["it_pcg"], ref.iters)
        assert info["relres_true"] <= 1e-8
        d = o.dbbd
        xr = np.empty(P.n)
        xr[np.concatenate([d.I, d.G])] = ref.w
        assert rel(x.cpu().numpy(), xr) < 1e-6
    finally:
        g.close()


def test_full_system_outer_batched_equals_alone():
    Ps = [PROBS["c1"](), PROBS["fd2d_40x36"]()]
    Ps[1].k, Ps[1].p = Ps[0].k, Ps[0].p
    probs, oms, bs = [], [], []
    for P in Ps:
        probs.append((torch.as_tensor(P.row_ptr, device="cuda"), torch.as_tensor(P.col, device="cuda"),
                      torch.as_tensor(P.val, device="cuda"), torch.as_tensor(P.part, device="cuda")))
        oms.append(dev(P.omega()))
        bs.append(dev(P.b()))
    h, _ = ns.nystrom_schur_setup_batched(probs, k=Ps[0].k, p=Ps[0].p, omegas=oms, outer=ns.NS_OUTER_FULL)
    try:
        xs, outs = ns.nystrom_schur_pcg_solve_batched(h, bs, rtol=1e-8, maxit=1000)
    finally:
        ns.nystrom_schur_destroy(h)
    for q, P in enumerate(Ps):
        g = gpu_setup(P, omega=P.omega(), k=Ps[0].k, p=Ps[0].p, outer=ns.NS_OUTER_FULL)
        try:
            x, info = g.solve(bs[q], rtol=1e-8, maxit=1000)
        finally:
            g.close()
        assert outs[q]["it_pcg"] == info["it_pcg"]
        assert rel(xs[q].cpu().numpy(), x.cpu().numpy()) < 1e-12


def test_batched_m1_power_equals_alone():
    Ps = [PROBS["c1"](), make_problem((40, 40), (2, 2), sigma=1.0, ell=4.0, k=20, p=10)]
    probs, oms = [], []
    for P in Ps:
        probs.append((torch.as_tensor(P.row_ptr, device="cuda"), torch.as_tensor(P.col, device="cuda"),
                      torch.as_tensor(P.val, device="cuda"), torch.as_tensor(P.part, device="cuda")))
        oms.append(dev(P.omega()))
    h, infos = ns.nystrom_schur_setup_batched(probs, k=20, p=10, omegas=oms, variant=ns.NS_VARIANT_M1, power_iters=1)
    try:
        for q, P in enumerate(Ps):
            g = gpu_setup(P, variant=ns.NS_VARIANT_M1, power_iters=1)
            try:
                assert infos[q]["it_inner"] == g.setup_info["it_inner"]
                assert infos[q]["k_eff"] == g.setup_info["k_eff"]
            finally:
                g.close()
    finally:
        ns.nystrom_schur_destroy(h)


def test_variant_option_errors():
    P = config_c1()
    with pytest.raises(ns.NsError) as e:
        gpu_setup(P, outer=ns.NS_OUTER_FULL, apply_mode=ns.NS_APPLY_ADEF2)
    assert e.value.status == ns.NS_ERR_INVALID_ARG
    with pytest.raises(ns.NsError) as e:
        gpu_setup(P, variant=7)
    assert e.value.status == ns.NS_ERR_INVALID_ARG
    with pytest.raises(ns.NsError) as e:
        gpu_setup(P, power_iters=-1)
    assert e.value.status == ns.NS_ERR_INVALID_ARG
    probs = [(torch.as_tensor(P.row_ptr, device="cuda"), torch.as_tensor(P.col, device="cuda"),
              torch.as_tensor(P.val, device="cuda"), torch.as_tensor(P.part, device="cuda"))] * 2
    om = dev(interior_sketch(P))
    with pytest.raises(ns.NsError) as e:
        ns.nystrom_schur_setup_batched(probs, k=P.k, p=P.p, omegas=[om, om], variant=ns.NS_VARIANT_M3)
    assert e.value.status == ns.NS_ERR_INVALID_ARG
