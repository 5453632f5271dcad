"""The learned engine switch: what the trained network gains over Eq. 3.

Regret (Sum(t_chosen - t_min) / Sum(t_min), following the paper's per-level
analysis of its switch) is computed for the learned and the Eq. 3 choices
from the SAME probe-mode timings, so the comparison does not depend on run to
run timing noise. Levels are exact regardless of the choices."""
import os

import numpy as np
import pytest

import oracle
from paper_2606_05081_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2606_05081_amd import blest, switch
    assert torch.cuda.is_available()
    return blest, switch


def test_small_training_run_beats_eq3_on_held_out_graph(env, capsys):
    blest, switch = env
    specs = [("rmat", 15, 4015), ("rmat", 16, 4016), ("rmat", 17, 4017), ("grid", 256, 4100), ("grid", 384, 4101)]
    X, T, H, fam = switch.build_dataset(specs, runs_per_graph=8, grid_levels_per_run=48, log=lambda *a: None)
    y = switch.labels_from_times(T, H)
    w = switch.cost_weights(T, fam)
    params, mean, std, losses = switch.train(X, y, w, steps=2000)
    assert losses[-100:].mean() < losses[:50].mean()
    ch = switch.predict(params, mean, std, X, switch.MIN_CONFIDENCE)
    ch = np.where(ch < 0, H, ch)
    r_train_l, r_train_h = switch.regret(T, ch), switch.regret(T, H)
    # held-out graph of the R-MAT family, seeds disjoint from training
    rp, col = inputs.rmat_graph(18, 4918)
    g = blest.Graph(rp, col)
    g.set_switch_model(params, mean, std, switch.MIN_CONFIDENCE)
    Xh, Th, Hh, _ = switch.probe_graph(g, inputs.sources(rp, 8, seed=4919))
    chh = switch.predict(params, mean, std, Xh, switch.MIN_CONFIDENCE)
    chh = np.where(chh < 0, Hh, chh)
    r_l, r_h = switch.regret(Th, chh), switch.regret(Th, Hh)
    with capsys.disabled():
        print(f"\n[switch] train regret learned {r_train_l:.4f} vs Eq.3 {r_train_h:.4f}; "
              f"held-out R-MAT s18 regret learned {r_l:.4f} vs Eq.3 {r_h:.4f}")
    assert r_train_l <= r_train_h + 1e-9
    assert r_l <= r_h + 0.02
    # the learned policy returns exact levels
    g.set_policy(blest.Policy.LEARNED)
    for s in inputs.sources(rp, 3, seed=4920):
        assert np.array_equal(g.bfs(int(s)).cpu().numpy(), oracle.bfs(rp, col, int(s)))
    g.close()


def test_committed_model_on_held_out_graphs(env, capsys):
    blest, switch = env
    if not os.path.exists(switch.MODEL_PATH):
        pytest.skip("no trained model committed yet (python -m paper_2606_05081_amd.switch)")
    params, mean, std, meta = switch.load_model()
    for kind, size, seed in [("rmat", 20, 4920), ("grid", 1024, 4921)]:
        rp, col = switch.make_graph(kind, size, seed)
        g = blest.Graph(rp, col)
        g.set_switch_model(params, mean, std, meta.get("min_confidence", 0.5))
        X, T, H, _ = switch.probe_graph(g, inputs.sources(rp, 4, seed=seed + 1), 64 if kind == "grid" else None)
        ch = switch.predict(params, mean, std, X, meta.get("min_confidence", 0.5))
        ch = np.where(ch < 0, H, ch)
        r_l, r_h = switch.regret(T, ch), switch.regret(T, H)
        with capsys.disabled():
            print(f"\n[switch] committed model on {kind}{size}: regret learned {r_l:.4f} vs Eq.3 {r_h:.4f}")
        assert r_l <= r_h + 0.02
        g.set_policy(blest.Policy.LEARNED)
        s = int(inputs.sources(rp, 1, seed=seed + 2)[0])
        assert np.array_equal(g.bfs(s).cpu().numpy(), oracle.bfs(rp, col, s))
        g.close()


def test_multi_source_committed_model_on_held_out_graphs(env, capsys):
    """The multi-source network (switch_model_ms.json) against the pairs rule
    on graphs outside its training set: probe regret from the same timings,
    end-to-end device time of both policies, and exact closeness with it."""
    blest, switch = env
    if not os.path.exists(switch.MS_MODEL_PATH):
        pytest.skip("no multi-source model committed yet (python -m paper_2606_05081_amd.switch --ms)")
    params, mean, std, meta = switch.load_model(switch.MS_MODEL_PATH)
    conf = meta.get("min_confidence", 0.5)
    for kind, size, seed in [("rmat", 20, 4930), ("grid", 640, 4931)]:
        rp, col = switch.make_graph(kind, size, seed)
        g = blest.Graph(rp, col)
        g.set_ms_switch_model(params, mean, std, conf)
        k, widths = switch.ms_width_plan(1)
        X, T, H, _ = switch.probe_ms(g, inputs.sources(rp, k, seed=seed + 1), widths)
        ch = switch.ms_predict(params, mean, std, X, conf)
        ch = np.where(ch < 0, H, ch)
        r_l, r_h = switch.regret(T, ch), switch.regret(T, H)
        srcs = inputs.sources(rp, 1024, seed=seed + 2)
        t_h = min(switch.ms_time(g, srcs, [512], blest.Policy.HEURISTIC) for _ in range(2))
        t_l = min(switch.ms_time(g, srcs, [512], blest.Policy.LEARNED) for _ in range(2))
        with capsys.disabled():
            print(f"\n[ms-switch] {kind}{size}: regret learned {r_l:.4f} vs pairs rule {r_h:.4f}; "
                  f"1024 sources {t_l:.2f} ms learned vs {t_h:.2f} ms pairs rule")
        assert r_l <= r_h + 0.02
        assert t_l <= t_h * 1.02
        cs = inputs.sources(rp, 96, seed=seed + 3)
        osum, oreach, occ = oracle.closeness(rp, col, cs)
        g.set_policy(blest.Policy.LEARNED)
        s_, r_, c_ = g.closeness(cs)
        assert np.array_equal(s_.cpu().numpy(), osum) and np.array_equal(r_.cpu().numpy(), oreach)
        assert np.array_equal(c_.cpu().numpy(), occ)
        g.close()
