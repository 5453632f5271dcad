"""Switch-network kernels (fp32, GPU) against the float64 oracle.

Tolerances: each gradient entry is a sum of at most batch products of
magnitude <= max|g|, so fp32 accumulation error is below batch * 2^-24 *
max|g| ~ 2e-5 max|g| for batch 300; the test allows rtol 1e-4 plus atol
1e-5 * max|g|."""
import math

import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2606_05081_amd import blest
    assert torch.cuda.is_available()
    return torch, blest


def dev(torch, a, dtype=None):
    return torch.tensor(np.asarray(a), device="cuda", dtype=dtype)


@pytest.mark.parametrize("batch,seed", [(1, 0), (127, 1), (128, 2), (300, 3), (1000, 4)])
def test_loss_grad_matches_float64_oracle(env, batch, seed):
    torch, blest = env
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.3, omlp.N_PARAMS)
    x = rng.normal(size=(batch, 12))
    y = rng.integers(0, 3, batch)
    w = rng.uniform(0.2, 3.0, batch)
    ref_loss, ref_g = omlp.loss_and_grad(theta, x, y, w)
    p32 = dev(torch, theta, torch.float32)
    loss = torch.zeros(1, device="cuda")
    grad = torch.zeros(omlp.N_PARAMS, device="cuda")
    blest.blest_mlp_loss_grad(p32, dev(torch, x, torch.float32), dev(torch, y, torch.int32),
                              dev(torch, w, torch.float32), loss, grad)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    # the oracle evaluated at the fp32-rounded inputs isolates kernel error from input rounding
    ref_loss32, ref_g32 = omlp.loss_and_grad(theta.astype(np.float32).astype(np.float64),
                                             x.astype(np.float32).astype(np.float64), y,
                                             w.astype(np.float32).astype(np.float64))
    assert abs(loss.item() - ref_loss32) <= 1e-5 * max(1.0, abs(ref_loss32))
    atol = 1e-5 * np.abs(ref_g32).max()
    assert np.all(np.abs(g - ref_g32) <= 1e-4 * np.abs(ref_g32) + atol), np.abs(g - ref_g32).max()
    assert abs(loss.item() - ref_loss) < 1e-3  # and close to the unrounded problem


def test_zero_weights_ln3(env):
    torch, blest = env
    x = np.random.default_rng(0).normal(size=(64, 12))
    y = np.arange(64) % 3
    loss = torch.zeros(1, device="cuda")
    grad = torch.zeros(omlp.N_PARAMS, device="cuda")
    blest.blest_mlp_loss_grad(torch.zeros(omlp.N_PARAMS, device="cuda"), dev(torch, x, torch.float32),
                              dev(torch, y, torch.int32), None, loss, grad)
    torch.cuda.synchronize()
    assert abs(loss.item() - math.log(3)) < 1e-6
    gb3 = grad.cpu().numpy()[-3:]
    exp = np.array([1 / 3 - np.mean(y == k) for k in range(3)])
    assert np.allclose(gb3, exp, atol=1e-7)


def test_forward_matches_oracle(env):
    torch, blest = env
    rng = np.random.default_rng(5)
    theta = rng.normal(0, 0.3, omlp.N_PARAMS)
    x = rng.normal(size=(777, 12))
    logits = torch.empty((777, 3), device="cuda")
    blest.blest_mlp_forward(dev(torch, theta, torch.float32), dev(torch, x, torch.float32), logits)
    torch.cuda.synchronize()
    ref, _ = omlp.forward(theta.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64))
    assert np.allclose(logits.cpu().numpy(), ref, rtol=1e-4, atol=1e-4 * np.abs(ref).max())


def test_adam_step_matches_oracle(env):
    torch, blest = env
    rng = np.random.default_rng(6)
    theta = rng.normal(0, 0.3, omlp.N_PARAMS)
    g = rng.normal(size=omlp.N_PARAMS)
    m0 = rng.normal(0, 0.01, omlp.N_PARAMS)
    v0 = rng.uniform(0, 0.01, omlp.N_PARAMS)
    p, gm, m, v = (dev(torch, a, torch.float32) for a in (theta, g, m0, v0))
    blest.blest_mlp_adam(p, gm, m, v, 7, lr=1e-3)
    torch.cuda.synchronize()
    # compare at fp32-rounded inputs and constants: in fp32, 1 - beta2 is
    # exactly 1 - fl32(0.999), which differs from 0.001 by 1.3e-5 relative
    r32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    t_ref, m_ref, v_ref = omlp.adam_step(r32(theta), r32(g), r32(m0), r32(v0), 7, lr=float(np.float32(1e-3)),
                                         beta1=float(np.float32(0.9)), beta2=float(np.float32(0.999)),
                                         eps=float(np.float32(1e-8)))
    assert np.allclose(p.cpu().numpy(), t_ref, rtol=1e-5, atol=1e-6)
    assert np.allclose(m.cpu().numpy(), m_ref, rtol=1e-5, atol=1e-7)
    assert np.allclose(v.cpu().numpy(), v_ref, rtol=1e-5, atol=1e-9)


def test_training_learns_a_separable_rule(env):
    torch, blest = env
    from paper_2606_05081_amd import switch
    rng = np.random.default_rng(7)
    X = rng.normal(size=(4000, 12)).astype(np.float32)
    y = np.where(X[:, 0] > 0.5, 2, np.where(X[:, 1] > 0, 1, 0)).astype(np.int32)
    w = np.ones(len(y), np.float32)
    params, mean, std, losses = switch.train(X, y, w, steps=1500, batch=256, lr=3e-3, seed=3)
    assert losses[-100:].mean() < 0.5 * losses[:20].mean()
    acc = (switch.predict(params, mean, std, X) == y).mean()
    assert acc > 0.9, acc


def test_in_kernel_inference_matches_oracle_decisions(env):
    torch, blest = env
    import oracle
    from paper_2606_05081_amd import inputs
    rng = np.random.default_rng(8)
    theta = rng.normal(0, 0.5, omlp.N_PARAMS).astype(np.float32)
    for rp, col in (inputs.rmat_graph(15, 9), inputs.grid_graph(64, 9)):
        # the lazy scheme runs every engine the network picks (the eager one runs push levels top-down)
        g = blest.Graph(rp, col, update_scheme=blest.Update.LAZY)
        feats = []
        for s in inputs.sources(rp, 3, seed=10):
            g.set_policy(blest.Policy.HEURISTIC)
            g.bfs(int(s))
            feats.append(g.level_features()[:-1])
        F = np.concatenate(feats)
        mean, std = F.mean(0), np.maximum(F.std(0), 1e-3)
        g.set_switch_model(theta, mean, std)
        g.set_policy(blest.Policy.LEARNED)
        for s in inputs.sources(rp, 3, seed=10):
            lev = g.bfs(int(s)).cpu().numpy()
            assert np.array_equal(lev, oracle.bfs(rp, col, int(s)))
            st = g.level_stats()
            f = g.level_features()
            for i, r in enumerate(st[:-1]):
                z = (f[i].astype(np.float64) - mean) / std.astype(np.float32)
                logit, _ = omlp.forward(theta.astype(np.float64), z[None, :])
                pr = np.exp(logit[0] - logit[0].max())
                pmax = 1.0 / pr.sum()
                if r["mlp_fallback"]:  # out of range, or below the default confidence floor 0.5
                    assert (np.abs(z) > 6 - 1e-4).any() or pmax < 0.5 + 1e-4
                    continue
                srt = np.sort(logit[0])
                if srt[-1] - srt[-2] < 1e-3 or abs(pmax - 0.5) < 1e-4:
                    continue  # near tie or at the floor: fp32 may decide either way
                assert r["engine"] == int(np.argmax(logit[0])), (i, logit)
        g.close()
