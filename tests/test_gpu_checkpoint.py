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
