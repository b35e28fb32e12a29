"""Learned starting subspace on the GPU: features, BF16 network forward and
gradient against the FP64 oracle, training, the Rayleigh-Ritz judge in setup
(accepted proposals deflate, rejected ones fall back to plain Nystrom
bit for bit), and what a trained network gains on held-out problems."""

import numpy as np
import pytest
import scipy.linalg as sla
import torch

import paper_2101_12164_amd as ns
from gpu_helpers import gpu_setup, to_dev
from oracle import NystromSchurOracle, dense_schur
from oracle import learned as L
from workloads import config_c1, make_problem

pytestmark = pytest.mark.gpu


def grid_coords(shape):
    idx = np.indices(shape).reshape(len(shape), -1).T[:, ::-1]  # x fastest, as the node numbering
    c = 2.0 * idx / np.maximum(np.array(shape[::-1]) - 1, 1) - 1.0
    out = np.zeros((idx.shape[0], 3))
    out[:, :c.shape[1]] = c
    return out


def features_gpu(P, coords):
    d = to_dev(P)
    return ns.nystrom_schur_features(d["row_ptr"], d["col"], d["val"], d["part"],
                                     torch.as_tensor(coords, device="cuda"))


def test_features_match_oracle():
    P = make_problem((14, 14, 14), (2, 2, 2), sigma=1.5, ell=4.0, k=4, p=2, field_seed=3)
    C = grid_coords(P.shape)
    Xg = features_gpu(P, C).cpu().numpy()
    Xo = L.interface_features(P.n, P.row_ptr, P.col, P.val, P.part, C)
    assert Xg.shape == Xo.shape == (P.n_gamma, 16)
    assert np.allclose(Xg, Xo.astype(np.float32), rtol=1e-6, atol=1e-6)


def make_net(d_in, h, k, seed):
    p = L.mlp_init(d_in, h, k, seed)
    rng = np.random.default_rng(seed + 1)
    for name in ("b1", "b2", "b3"):
        p[name] = 0.05 * rng.standard_normal(p[name].shape)
    return p


def bf16(a):
    """Round float64 values to bfloat16 (nearest even) and back."""
    t = torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.to(torch.float64).numpy()


def emulated_forward(p32, X):
    """The network as the GPU evaluates it: BF16 inputs, weights and hidden activations, exact sums."""
    q = dict(p32)
    for name in ("W1", "W2", "W3"):
        q[name] = bf16(p32[name])
    Xb = bf16(X)
    A1 = Xb @ q["W1"] + q["b1"]
    H1 = bf16(np.maximum(A1, 0.0))
    A2 = H1 @ q["W2"] + q["b2"]
    H2 = bf16(np.maximum(A2, 0.0))
    Z0 = H2 @ q["W3"] + q["b3"]
    return Z0, q, (Xb, A1, H1, A2, H2)


def c4_features():
    """Features of the 48^3 lognormal family member 0 (sigma 1.5, 3^3 boxes): the learned layer's input at
    full size, from the oracle's feature routine."""
    from workloads import config_c4

    P = config_c4(seed=0)
    X = L.interface_features(P.n, P.row_ptr, P.col, P.val, P.part, grid_coords(P.shape))
    return X.astype(np.float32)


@pytest.mark.parametrize("case", ["small", "c4_full"])
def test_forward_and_gradient_match_oracle(case):
    rng = np.random.default_rng(0)
    if case == "small":
        n, d_in, h, k = 700, 16, 64, 8
        X = rng.standard_normal((n, d_in)).astype(np.float32)
    else:
        # the full-size configuration: 13 256 interface nodes, network 16 -> 256 -> 256 -> 48
        X = c4_features()
        n, d_in, h, k = X.shape[0], 16, 256, 48
    p = make_net(d_in, h, k, 11)
    flat = L.flatten(p).astype(np.float32)
    p32 = L.unflatten(flat.astype(np.float64), d_in, h, k)
    U = np.linalg.qr(rng.standard_normal((n, k)))[0]
    m = ns.nystrom_schur_mlp_create(d_in, h, k, flat)
    try:
        Xd = torch.as_tensor(X, device="cuda")
        Z0 = ns.nystrom_schur_mlp_forward(m, Xd, k).cpu().numpy()
        Zo, cache = L.mlp_forward(p32, X.astype(np.float64))
        Ze, qe, ce = emulated_forward(p32, X.astype(np.float64))
        # the kernels against the same roundings, then the BF16 cost against the FP64 network
        assert np.linalg.norm(Z0 - Ze) <= 1e-4 * np.linalg.norm(Ze)
        assert np.linalg.norm(Z0 - Zo) <= 1e-2 * np.linalg.norm(Zo)
        loss = ns.nystrom_schur_mlp_loss_grad(m, Xd, torch.as_tensor(U, device="cuda"))
        assert abs(loss - L.subspace_loss(Ze, U)) <= 1e-4 * L.subspace_loss(Ze, U)
        lo = L.subspace_loss(Zo, U)
        assert abs(loss - lo) <= 1e-2 * max(lo, 1e-3)
        _, g = ns.nystrom_schur_mlp_get_params(m, flat.size)
        gg = L.unflatten(g.astype(np.float64), d_in, h, k)
        ge = L.mlp_backward(qe, ce, L.subspace_loss_grad(Ze, U))
        go = L.mlp_backward(p32, cache, L.subspace_loss_grad(Zo, U))
        for name in L.PARAM_ORDER:
            nrm = lambda a: max(np.linalg.norm(a), 1e-30)  # noqa: E731
            ee = np.linalg.norm(gg[name] - ge[name]) / nrm(ge[name])
            eo = np.linalg.norm(gg[name] - go[name]) / nrm(go[name])
            cos = float(np.sum(gg[name] * go[name]) / (nrm(gg[name]) * nrm(go[name])))
            print(name, "vs BF16-emulated", ee, "vs FP64", eo, "cosine", cos, flush=True)
            # the kernels compute exactly the BF16-rounded network; the distance to the FP64 network's
            # gradient is the BF16 rounding amplified by the conditioning of G = Z0^T Z0 at this random init
            # (FP32 backward over 13 256 rows at full size: 6e-3 measured for W3)
            assert ee <= (5e-3 if case == "small" else 1e-2), name
            # at full size the BF16 rounding of the features and hidden activations moves the gradients of the
            # first two layers by about a third against the FP64 network (measured 0.34, 0.31, 0.35 for W1, b1,
            # W2, cosines 0.94-0.95); the kernels still match the BF16-rounded network to 5e-3
            eo_max, cos_min = (1e-1, 0.99) if case == "small" else (0.5, 0.9)
            assert eo <= eo_max and cos >= cos_min, name
    finally:
        ns.nystrom_schur_mlp_destroy(m)


def test_training_lowers_the_loss():
    rng = np.random.default_rng(1)
    n, d_in, h, k = 900, 16, 64, 6
    X = rng.standard_normal((n, d_in)).astype(np.float32)
    # a target subspace the network can represent: smooth functions of the first features
    B = np.stack([np.sin(X[:, 0] * (j + 1)) + X[:, 1] * j for j in range(k)], axis=1)
    U = np.linalg.qr(B.astype(np.float64))[0]
    m = ns.nystrom_schur_mlp_create(d_in, h, k, L.flatten(make_net(d_in, h, k, 5)).astype(np.float32))
    try:
        Xd, Ud = torch.as_tensor(X, device="cuda"), torch.as_tensor(U, device="cuda")
        first = ns.nystrom_schur_mlp_loss_grad(m, Xd, Ud)
        for _ in range(150):
            ns.nystrom_schur_mlp_loss_grad(m, Xd, Ud)
            ns.nystrom_schur_mlp_adam_step(m, 3e-3)
        last = ns.nystrom_schur_mlp_loss_grad(m, Xd, Ud)
        print("loss", first, "->", last, flush=True)
        assert last < 0.5 * first
    finally:
        ns.nystrom_schur_mlp_destroy(m)


def exact_proposal(P, k):
    orc = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=0, p=0, omega=None)
    d = orc.dbbd
    S = dense_schur(d)
    AG = d.A_G.toarray()
    lam, V = sla.eigh(S, AG)
    return AG @ V[:, :k]


def test_exact_proposal_is_accepted():
    P = config_c1()
    Z0 = exact_proposal(P, P.k)
    b = torch.as_tensor(P.b(), device="cuda")
    h = gpu_setup(P, proposal=torch.as_tensor(Z0, device="cuda"))
    try:
        assert h.setup_info["proposal_accepted"] == 1 and h.setup_info["it_inner"] == 0
        _, rho = ns.nystrom_schur_get_basis(h.handle)
        assert rho <= 1e-8
        x, out = h.solve(b, rtol=1e-8)
    finally:
        h.close()
    o = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=P.k, p=P.p, omega=P.omega(), proposal=Z0)
    so = o.solve(P.b())
    assert o.setup_result.proposal_accepted
    assert abs(out["it_pcg"] - so.it_pcg) <= 1
    assert out["relres_true"] <= 1e-8


def test_rejected_proposal_falls_back_bitwise():
    P = config_c1()
    Z0 = np.random.default_rng(2).standard_normal((P.n_gamma, P.k))
    b = torch.as_tensor(P.b(), device="cuda")
    h1 = gpu_setup(P, proposal=torch.as_tensor(Z0, device="cuda"))
    h0 = gpu_setup(P)
    try:
        assert h1.setup_info["proposal_accepted"] == 0
        assert h1.setup_info["it_inner"] == h0.setup_info["it_inner"]
        x1, o1 = h1.solve(b)
        x0, o0 = h0.solve(b)
        assert o1["it_pcg"] == o0["it_pcg"] and torch.equal(x1, x0)
    finally:
        h1.close()
        h0.close()


def family(seed, N=20):
    P = make_problem((N, N, N), (2, 2, 2), sigma=1.5, ell=6.0, field_seed=seed, k=8, p=4, seed=seed,
                     name=f"logn3d_{N}_{seed}")
    return P, grid_coords(P.shape)


def test_trained_network_gain_on_held_out_problems():
    """Train on a small family (3D lognormal sigma 1.5, 2x2x2 subdomains) with the bases the method itself
    produces, then judge the network's proposals on held-out seeds.  Every held-out solve converges
    (accepted proposals deflate, rejected ones fall back); the acceptance rate and the change in setup time
    and PCG iterations are what the network gains."""
    k, h = 8, 128
    train = [family(s) for s in range(12)]
    held = [family(1000 + s) for s in range(4)]
    data = []
    for P, C in train:
        hs = gpu_setup(P)
        U, _ = ns.nystrom_schur_get_basis(hs.handle)
        hs.close()
        data.append((features_gpu(P, C), U.contiguous()))
    m = ns.nystrom_schur_mlp_create(16, h, k, L.flatten(make_net(16, h, k, 7)).astype(np.float32))
    try:
        losses = []
        for ep in range(25):
            tot = 0.0
            for X, U in data:
                tot += ns.nystrom_schur_mlp_loss_grad(m, X, U)
                ns.nystrom_schur_mlp_adam_step(m, 2e-3)
            losses.append(tot / len(data))
        print("training loss", [round(v, 3) for v in losses[::5]], round(losses[-1], 3), flush=True)
        assert losses[-1] < losses[0]
        acc = 0
        for P, C in held:
            X = features_gpu(P, C)
            Z0 = ns.nystrom_schur_mlp_forward(m, X, k)
            b = torch.as_tensor(P.b(), device="cuda")
            hl = gpu_setup(P, proposal=Z0)
            hp = gpu_setup(P)
            try:
                _, rho = ns.nystrom_schur_get_basis(hl.handle)
                xl, ol = hl.solve(b)
                xp, op = hp.solve(b)
                a = hl.setup_info["proposal_accepted"]
                acc += a
                print(P.name, "accepted", a, "rho", round(rho, 3), "it_pcg learned/plain", ol["it_pcg"],
                      op["it_pcg"], "setup s", round(hl.setup_info["t_total"], 4), round(hp.setup_info["t_total"], 4),
                      flush=True)
                assert ol["relres_true"] <= 1e-8 and op["relres_true"] <= 1e-8
                if not a:
                    assert ol["it_pcg"] == op["it_pcg"]
            finally:
                hl.close()
                hp.close()
        print("accepted", acc, "of", len(held), flush=True)
    finally:
        ns.nystrom_schur_mlp_destroy(m)
