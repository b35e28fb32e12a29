"""GPU: block-CG iterations replayed from a HIP graph give the same inner solve as plain launches -- the same
it_SI, and bit for bit the same low-rank term and preconditioner -- alone and batched, in FP64, FP32 and BF16,
for graphs of 2 and 4 iterations (iterations a replay runs after convergence change nothing)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2101_12164_amd as ns  # noqa: E402
from gpu_helpers import gpu_setup  # noqa: E402
from workloads import config_c1, make_problem  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


PROBS = {
    "c1": lambda: config_c1(),
    "lognormal2d_128": lambda: make_problem((128, 128), (4, 4), sigma=2.0, ell=8.0, k=32, p=8),
    "lognormal3d_24": lambda: make_problem((24, 24, 24), (2, 2, 2), sigma=2.0, ell=6.0, k=24, p=8),
}


@pytest.mark.parametrize("prec", [ns.NS_FP64, ns.NS_FP32, ns.NS_BF16])
@pytest.mark.parametrize("name", sorted(PROBS))
def test_graph_bcg_equals_plain_launches(name, prec):
    P = PROBS[name]()
    R = dev(np.random.default_rng(3).standard_normal((P.n_gamma, 3)))
    out = {}
    for mode in (-1, 2, 4):
        h = gpu_setup(P, prec_inner=prec, bcg_graph_iters=mode)
        try:
            Z, S = ns.nystrom_schur_get_lowrank(h.handle)
            out[mode] = (h.setup_info["it_inner"], h.setup_info["k_eff"], Z.clone(), S.clone(), h.apply(R).clone())
        finally:
            h.close()
    print(f"[graph-bcg] {name} prec={prec}: it_SI {out[-1][0]}", flush=True)
    for mode in (2, 4):
        assert out[mode][0] == out[-1][0] and out[mode][1] == out[-1][1]
        for a, b in zip(out[mode][2:], out[-1][2:]):
            assert torch.equal(a, b)


def test_graph_bcg_batched_equals_plain_launches():
    Ps = [PROBS["c1"](), make_problem((40, 40), (2, 2), sigma=1.0, ell=4.0, k=20, p=10),
          make_problem((64, 48), (3, 2), sigma=2.0, ell=6.0, k=20, p=10)]
    probs = [(torch.as_tensor(P.row_ptr, device="cuda"), torch.as_tensor(P.col, device="cuda"),
              torch.as_tensor(P.val, device="cuda"), torch.as_tensor(P.part, device="cuda")) for P in Ps]
    oms = [dev(P.omega()) for P in Ps]
    ng = sum(P.n_gamma for P in Ps)
    R = dev(np.random.default_rng(4).standard_normal((ng, 2)))
    res = {}
    for mode in (-1, 2):
        h, infos = ns.nystrom_schur_setup_batched(probs, k=20, p=10, omegas=oms, bcg_graph_iters=mode)
        try:
            res[mode] = ([i["it_inner"] for i in infos], ns.nystrom_schur_apply(h, R).clone())
        finally:
            ns.nystrom_schur_destroy(h)
    assert res[2][0] == res[-1][0]
    assert torch.equal(res[2][1], res[-1][1])
