"""GPU: the tuned-settings table (paper_2101_12164_amd/tuning_gfx950.tsv, written by the autotuner) is loaded
beside the library, the values it gives a handle are reported, explicit options and process-wide overrides
take precedence, and every candidate value of every tuned setting gives the same results."""

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


def table_entries():
    path = ns.library_path().rsplit("/", 1)[0] + "/tuning_gfx950.tsv"
    out = []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        arch, kernel, prec, lo, hi, v = line.split()
        out.append((kernel, prec, int(lo), int(hi), int(v)))
    return out


def lookup(kernel, prec, size, default):
    for k, p, lo, hi, v in table_entries():
        if k == kernel and p in ("*", prec) and lo <= size <= hi:
            return v
    return default


def test_table_loaded_and_reported():
    n, path = ns.nystrom_schur_tuning_info()
    assert n == len(table_entries()) > 0 and path.endswith("tuning_gfx950.tsv")
    P = config_c1()
    g = gpu_setup(P)
    try:
        t = ns.nystrom_schur_get_tuning(g.handle)
        s = P.k + P.p
        assert t["trsm_cols"] == lookup("trsm_cols", "f64", s, 32)
        assert t["pcg_graph_iters"] == lookup("pcg_graph_iters", "f64", P.n_gamma, 1)
        assert t["bcg_graph_iters"] == lookup("bcg_graph_iters", "f64", P.n_gamma, 2)
    finally:
        g.close()
    # explicit options and overrides take precedence
    g = gpu_setup(P, pcg_graph_iters=8, trsm_cols=64)
    try:
        t = ns.nystrom_schur_get_tuning(g.handle)
        assert t["pcg_graph_iters"] == 8 and t["trsm_cols"] == 64
    finally:
        g.close()
    ns.nystrom_schur_tuning_override("bcg_graph_iters", 6)
    try:
        g = gpu_setup(P)
        assert ns.nystrom_schur_get_tuning(g.handle)["bcg_graph_iters"] == 6
        g.close()
    finally:
        ns.nystrom_schur_tuning_override("bcg_graph_iters", 0)


@pytest.mark.parametrize("maker", [lambda: config_c1(),
                                   lambda: make_problem((32, 32, 32), (2, 2, 2), sigma=2.0, ell=8.0, k=64, p=16)])
def test_every_candidate_gives_the_same_result(maker):
    P = maker()
    b = dev(P.b())

    def run(**kw):
        g = gpu_setup(P, **kw)
        try:
            x, info = g.solve(b, rtol=1e-8, maxit=2000)
            return g.setup_info["it_inner"], info["it_pcg"], x.clone()
        finally:
            g.close()

    ref = run()
    cases = [dict(pcg_graph_iters=v) for v in (1, 2, 4, 8)] + [dict(bcg_graph_iters=v) for v in (2, 4, 8)]
    cases += [dict(trsm_cols=v, schur_mode=ns.NS_SCHUR_TRIANGULAR) for v in (16, 32, 64)]
    tri = run(schur_mode=ns.NS_SCHUR_TRIANGULAR)
    for kw in cases:
        r = run(**kw)
        base = tri if "trsm_cols" in kw else ref
        assert r[0] == base[0] and r[1] == base[1], kw
        assert float(torch.linalg.norm(r[2] - base[2]) / torch.linalg.norm(base[2])) <= 1e-12, kw
    for v in (64, 80):
        ns.nystrom_schur_tuning_override("ls_gemm_cols", v)
        try:
            r = run()
        finally:
            ns.nystrom_schur_tuning_override("ls_gemm_cols", 0)
        assert r[0] == ref[0] and r[1] == ref[1]
        assert float(torch.linalg.norm(r[2] - ref[2]) / torch.linalg.norm(ref[2])) <= 1e-12
