"""GPU: the inner system exactly as Algorithm alg:prec1 step 3 prints it (NS_INNER_FORM_A): block CG on
S_I X = A_IGamma G over the interior rows, preconditioned by A_I^{-1}, then B G = A_GammaI X (for M_3:
S_I X = G), against the FP64 oracle's inner='formA' run with the same sketch: it_SI and it_PCG within one,
k_eff equal, M r element by element, the 1e-8 true residual; unsupported combinations rejected."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2101_12164_amd as ns  # noqa: E402
from gpu_helpers import gpu_setup, oracle, rel  # noqa: E402
from workloads import config_c1, make_problem  # noqa: E402

PROBS = {
    "c1": lambda: config_c1(),
    "lognormal2d_96": lambda: make_problem((96, 96), (3, 3), sigma=2.0, ell=8.0, k=24, p=8),
    "fd3d_14": lambda: make_problem((14, 14, 14), (2, 2, 2), sigma=0.0, ell=8.0, k=10, p=5),
}


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def interior_sketch(P):
    nI = int(np.count_nonzero(P.part >= 0))
    return np.random.default_rng(100 + P.seed).standard_normal((nI, P.k + P.p))


CASES = [(p, v, m) for p in sorted(PROBS) for v in ("M2", "M3") for m in ("M2", "ADEF2")]


@pytest.mark.parametrize("pname,variant,mode", CASES, ids=[f"{a}-{b}-{c}" for a, b, c in CASES])
def test_form_a_matches_oracle(pname, variant, mode):
    P = PROBS[pname]()
    om = interior_sketch(P) if variant == "M3" else P.omega()
    print(f"[form A] {pname} variant={variant} mode={mode}", flush=True)
    o = oracle(P, variant=variant, apply_mode=mode, omega=om, inner="formA")
    r = o.solve(P.b(), tol=1e-8)
    g = gpu_setup(P, omega=om, variant={"M2": ns.NS_VARIANT_M2, "M3": ns.NS_VARIANT_M3}[variant],
                  apply_mode={"M2": ns.NS_APPLY_M2, "ADEF2": ns.NS_APPLY_ADEF2}[mode], inner_form=ns.NS_INNER_FORM_A)
    try:
        si = g.setup_info
        x, info = g.solve(dev(P.b()), rtol=1e-8, maxit=2000)
        R = np.random.default_rng(3).standard_normal((o.dbbd.n_gamma, 3))
        em = rel(ns.nystrom_schur_apply(g.handle, dev(R)).cpu().numpy(), o.apply(R))
        print(f"[form A] it_SI {si['it_inner']} (oracle {o.setup_result.it_inner}), k_eff {si['k_eff']} "
              f"(oracle {o.setup_result.k_eff}), it_PCG {info['it_pcg']} (oracle {r.it_pcg}), relres_true "
              f"{info['relres_true']:.2e}, M r error {em:.2e}", flush=True)
        assert abs(si["it_inner"] - o.setup_result.it_inner) <= 1
        assert si["k_eff"] == o.setup_result.k_eff
        assert abs(info["it_pcg"] - r.it_pcg) <= 1
        assert info["relres_true"] <= 1e-8
        assert em < 1e-7
    finally:
        g.close()


def test_form_a_and_shifted_build_the_same_product():
    """With a tight inner tolerance both inner systems give the same B G (eq. S-1), so the two preconditioners
    coincide to the solve accuracy."""
    P = PROBS["lognormal2d_96"]()
    R = dev(np.random.default_rng(8).standard_normal((P.n_gamma, 2)))
    z = []
    for form in (ns.NS_INNER_SHIFTED, ns.NS_INNER_FORM_A):
        g = gpu_setup(P, tol_inner=1e-12, inner_form=form, max_inner_iters=500)
        try:
            z.append(ns.nystrom_schur_apply(g.handle, R).cpu().numpy())
        finally:
            g.close()
    assert rel(z[1], z[0]) < 1e-7


def test_form_a_rejections():
    P = PROBS["c1"]()
    for kw in (dict(prec_inner=ns.NS_FP32), dict(prec_inner=ns.NS_BF16), dict(variant=ns.NS_VARIANT_M1)):
        with pytest.raises(ns.NsError):
            gpu_setup(P, inner_form=ns.NS_INNER_FORM_A, **kw)
    with pytest.raises(ns.NsError):
        gpu_setup(P, inner_form=7)
