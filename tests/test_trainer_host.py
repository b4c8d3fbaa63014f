"""Host logic of the warm-start trainer (no GPU): its checkpoint format."""


def test_training_checkpoint_roundtrip(tmp_path):
    """The trainer's checkpoint holds parameters, Adam moments, the step and the
    minibatch generator's state: reloading it continues the same sequence."""
    import numpy as np
    import torch
    from paper_2602_19697_amd import learned
    rng = np.random.default_rng(3)
    p, m, v = (torch.from_numpy(rng.standard_normal(50).astype(np.float32)) for _ in range(3))
    mb = np.random.default_rng(7)
    mb.integers(0, 100, size=5)
    path = str(tmp_path / "ck.npz")
    learned.save_checkpoint(path, p, m, v, 42, mb, [(1, 0.5), (40, 0.25)])
    p2, m2, v2, step, state, hist = learned.load_checkpoint(path)
    assert np.array_equal(p2, p.numpy()) and np.array_equal(m2, m.numpy()) and np.array_equal(v2, v.numpy())
    assert step == 42 and hist == [(1, 0.5), (40, 0.25)]
    again = np.random.default_rng(0)
    again.bit_generator.state = state
    assert np.array_equal(again.integers(0, 100, size=8), mb.integers(0, 100, size=8))
