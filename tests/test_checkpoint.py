"""Checkpoints of the learned-shadow network (no GPU needed: the file format and its
checks).  The trainer's checkpoints are exercised on the GPU in test_gpu_train.py."""
import numpy as np
import pytest
import torch

from paper_2606_28581_amd import surrogate as sg


def test_network_checkpoint_round_trip(tmp_path):
    rng = np.random.default_rng(4)
    w, m, v = (torch.as_tensor(rng.standard_normal(sg.N_PARAMS).astype(np.float32)) for _ in range(3))
    path = tmp_path / "net.npz"
    sg.save_network(path, (1.5, -2.0, 3.25), 0.125, w, m, v, step=37)
    d = sg.load_network(path, device="cpu")
    assert d["step"] == 37 and d["inv_half"] == 0.125
    np.testing.assert_array_equal(d["centre"], [1.5, -2.0, 3.25])
    for k, t in (("w", w), ("m", m), ("v", v)):
        assert torch.equal(d[k], t), k
    # weights only (inference)
    sg.save_network(path, (0, 0, 0), 1.0, w)
    d = sg.load_network(path, device="cpu")
    assert d["m"] is None and d["v"] is None and d["step"] == 0
    assert torch.equal(d["w"], w)


def test_network_checkpoint_rejects_wrong_sizes(tmp_path):
    with pytest.raises(ValueError):
        sg.save_network(tmp_path / "a.npz", (0, 0, 0), 1.0, np.zeros(sg.N_PARAMS - 1, np.float32))
    with pytest.raises(ValueError):
        sg.save_network(tmp_path / "b.npz", (0, 0, 0), 1.0, np.zeros(sg.N_PARAMS, np.float32),
                        m=np.zeros(sg.N_PARAMS, np.float32))
    np.savez(tmp_path / "c.npz", centre=np.zeros(3), inv_half=np.float64(1), step=np.int64(0),
             w=np.zeros(5, np.float32))
    with pytest.raises(ValueError):
        sg.load_network(tmp_path / "c.npz", device="cpu")
