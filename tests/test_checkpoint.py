"""Checkpoint and resume (host-side, no GPU): the surrogate's weights, Adam moments and step
count, its input statistics and threshold, and the inverse problem's optimiser state all
survive a save and load exactly, through the safe tensor-only loader."""

import numpy as np
import torch


def test_surrogate_checkpoint_round_trip(tmp_path):
    from paper_2511_09389_amd.surrogate import Surrogate, SurrogateNet
    net = SurrogateNet(torch.device("cpu"), seed=3)
    g = torch.Generator().manual_seed(1)
    for t in net.m + net.v + net.w + net.b:
        t.copy_(torch.randn(t.shape, generator=g))
    net.step = 17
    model = Surrogate(net, np.arange(6, dtype=np.float32) + 0.5, threshold=0.0125)
    path = tmp_path / "surrogate.pt"
    model.save(path)
    back = Surrogate.load(path, torch.device("cpu"))
    assert back.net.step == 17
    assert back.threshold == 0.0125
    assert np.array_equal(back.stats, model.stats)
    for a, b in zip(net.w + net.b + net.m + net.v, back.net.w + back.net.b + back.net.m + back.net.v):
        assert torch.equal(a, b)
    for a, b in zip(net.w, back.net.wb):   # the bf16 copies the kernels read follow the masters
        assert torch.equal(a.to(torch.bfloat16), b)


def test_inverse_state_round_trip(tmp_path):
    from paper_2511_09389_amd.inverse import InverseState
    g = torch.Generator().manual_seed(2)
    st = InverseState(torch.randn((5, 6, 7), generator=g), torch.randn((5, 6, 7), generator=g),
                      torch.rand((5, 6, 7), generator=g), 42, [3.0, 2.5, 1.25])
    path = tmp_path / "inverse.pt"
    st.save(path)
    back = InverseState.load(path, torch.device("cpu"))
    assert back.step == 42 and back.losses == [3.0, 2.5, 1.25]
    for a, b in ((st.j, back.j), (st.m, back.m), (st.v, back.v)):
        assert torch.equal(a, b)
