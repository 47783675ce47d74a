"""Checkpoint and restore of the committed state, and network files: a restored
simulation continues bitwise as the saved one (Broyden histories end with each
step, so the committed state is the whole state); mismatched files are refused."""
import numpy as np
import pytest

from paper_1903_12609_amd import synth

pytestmark = pytest.mark.gpu


def _sim(w, graph=0):
    import paper_1903_12609_amd as fil
    return fil.Sim(w.fil_off, w.Y, w.q, w.params, graph=graph)


@pytest.mark.parametrize("graph", [0, 4])
def test_restore_continues_identically(tmp_path, graph):
    print("case checkpoint graph", graph, flush=True)
    w = synth.sediment_suspension(M=8, N=20, side=60.0, seed=31, dt_over_T=1 / 30)
    a = _sim(w, graph)
    for _ in range(4):
        a.step()
    path = tmp_path / "sim.ckpt"
    a.checkpoint(path)
    ra = [a.step()[0]["iters"] for _ in range(3)]
    Ya, qa, Xa = a.read_state()
    b = _sim(w, graph)
    b.restore(path)
    rb = [b.step()[0]["iters"] for _ in range(3)]
    Yb, qb, Xb = b.read_state()
    assert ra == rb
    assert np.array_equal(Ya, Yb) and np.array_equal(qa, qb) and np.array_equal(Xa, Xb)
    assert a.time_step() == b.time_step()
    a.close()
    b.close()


def test_restore_refuses_other_layout_and_garbage(tmp_path):
    import paper_1903_12609_amd as fil
    w1 = synth.sediment_suspension(M=8, N=20, side=60.0, seed=31, dt_over_T=1 / 30)
    w2 = synth.sediment_suspension(M=8, N=21, side=60.0, seed=31, dt_over_T=1 / 30)
    a, b = _sim(w1), _sim(w2)
    a.step()
    path = tmp_path / "sim.ckpt"
    a.checkpoint(path)
    Y0, q0, X0 = b.read_state()
    with pytest.raises(fil.FilError):
        b.restore(path)
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(b"not a checkpoint at all")
    with pytest.raises(fil.FilError):
        a.restore(bad)
    with pytest.raises(fil.FilError):
        a.restore(tmp_path / "missing.ckpt")
    Y1, q1, X1 = b.read_state()
    assert np.array_equal(Y0, Y1) and np.array_equal(X0, X1)
    a.close()
    b.close()


def test_network_file_round_trip(tmp_path):
    import paper_1903_12609_amd as fil
    import torch
    m1 = fil.MLP(8, width=64, depth=2, max_batch=64, seed=1)
    m2 = fil.MLP(8, width=64, depth=2, max_batch=32, seed=2)
    path = tmp_path / "net.bin"
    m1.save(path)
    m2.load(path)
    assert np.array_equal(m1.get_params(), m2.get_params())
    assert np.array_equal(m1.get_norm(), m2.get_norm())
    rng = np.random.default_rng(3)
    feat = torch.from_numpy(rng.standard_normal((16, m1.n_in)).astype(np.float32)).cuda()
    xb, _ = m1.standardize(feat)
    assert torch.equal(m1.forward(xb), m2.forward(xb))
    m3 = fil.MLP(8, width=32, depth=2, max_batch=64, seed=1)
    with pytest.raises(fil.FilError):
        m3.load(path)
    for m in (m1, m2, m3):
        m.close()


def _cilia(graph):
    import paper_1903_12609_amd as fil
    import cilia_cases as cc
    fo, Y, q, p = cc.pair()
    g = fil.Sim(fo, Y, q, p, graph=graph)
    g.set_wall()
    g.set_geometric_switch(cc.AXIS, cc.NORMAL, cc.THETA_MAX, cc.TAU_POS, cc.TAU_NEG, cc.N_TR)
    return g


@pytest.mark.parametrize("graph", [0, 8])
def test_restore_continues_switch_driven_cilia(tmp_path, graph):
    """Two pinned cilia on the wall driven by the geometric switch: the checkpoint is taken
    one step after the first reversal, inside the torque's transition, so the restored run
    matches only if the switch's direction, age and torque come back with the state."""
    print("case checkpoint cilia graph", graph, flush=True)
    a = _cilia(graph)
    for j in range(60):
        a.step()
        if (a.read_switch() < 0).any():
            break
    assert (a.read_switch() < 0).any(), "no reversal within 60 steps"
    a.step()
    path = tmp_path / "cilia.ckpt"
    a.checkpoint(path)
    ra = [a.step()[0]["iters"] for _ in range(8)]
    da = a.read_switch()
    Ya, qa, Xa = a.read_state()
    b = _cilia(graph)
    b.restore(path)
    rb = [b.step()[0]["iters"] for _ in range(8)]
    assert ra == rb
    assert np.array_equal(da, b.read_switch())
    Yb, qb, Xb = b.read_state()
    assert np.array_equal(Ya, Yb) and np.array_equal(qa, qb) and np.array_equal(Xa, Xb)
    # a simulation without the switch refuses the file, and a switch-driven one refuses a
    # file without switch state; neither is changed
    import paper_1903_12609_amd as fil
    import cilia_cases as cc
    fo, Y, q, p = cc.pair()
    c = fil.Sim(fo, Y, q, p)
    c.set_wall()
    with pytest.raises(fil.FilError):
        c.restore(path)
    c.checkpoint(tmp_path / "plain.ckpt")
    with pytest.raises(fil.FilError):
        b.restore(tmp_path / "plain.ckpt")
    assert np.array_equal(Yb, b.read_state()[0])
    for s in (a, b, c):
        s.close()


def test_setter_after_failed_first_step_drops_captured_blocks():
    """The 6 x 6 array of clamped, curvature-driven filaments fails its first step in
    unbounded fluid (the block-diagonal J0 misses the tether monopoles' coupling) and
    converges above the wall.  A first step that fails with graph blocks captured, then
    fil_set_wall, then steps: the blocks captured with the unbounded mobility must not be
    replayed, so the run equals one that set the wall before stepping."""
    import paper_1903_12609_amd as fil
    w = synth.active_array(nx=6, ny=6, N=20, spacing=20.0, seed=1003, base_z=synth.DL)
    a = fil.Sim(w.fil_off, w.Y, w.q, w.params, graph=8)
    r = a.step(raise_on_fail=False)
    assert isinstance(r, tuple) and not r[1][0]["converged"]
    a.set_wall()
    c = fil.Sim(w.fil_off, w.Y, w.q, w.params, graph=0)
    c.set_wall()
    for j in range(3):
        ra, rc_ = a.step()[0], c.step()[0]
        assert ra["iters"] == rc_["iters"] and ra["converged"], (j, ra, rc_)
    assert np.array_equal(a.read_state()[0], c.read_state()[0])
    assert np.array_equal(a.read_state()[2], c.read_state()[2])
    a.close()
    c.close()
