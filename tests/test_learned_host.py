"""Host-only checks of the learned filter's training state: a checkpoint
written by LearnedDecimation.save_checkpoint restores the master weights, both
AdamW moments, the step count and the hyper-parameters exactly."""

import numpy as np
import pytest
import torch

import paper_1708_07515_amd as pkg
from paper_1708_07515_amd._lib import LEARNED_PARAMS


def test_checkpoint_round_trip(tmp_path):
    net = pkg.LearnedDecimation("cpu", seed=3, lr=7e-4, betas=(0.8, 0.99), eps=1e-7, weight_decay=0.01)
    gen = torch.Generator().manual_seed(1)
    net.load(torch.randn(LEARNED_PARAMS, generator=gen))
    net.m1.copy_(torch.randn(LEARNED_PARAMS, generator=gen))
    net.m2.copy_(torch.rand(LEARNED_PARAMS, generator=gen))
    net.step_count = 41
    path = tmp_path / "ck.npz"
    net.save_checkpoint(path)
    other = pkg.LearnedDecimation("cpu", seed=9)
    other.load_checkpoint(path)
    for a, b in ((net.master, other.master), (net.m1, other.m1), (net.m2, other.m2)):
        assert torch.equal(a, b)
    assert torch.equal(other.weights, net.master.to(torch.bfloat16))
    assert other.step_count == 41
    assert (other.lr, other.betas, other.eps, other.weight_decay) == (7e-4, (0.8, 0.99), 1e-7, 0.01)


def test_checkpoint_refuses_other_files(tmp_path):
    path = tmp_path / "bad.npz"
    with open(path, "wb") as f:
        np.savez(f, master=np.zeros(10, np.float32), m1=np.zeros(10, np.float32), m2=np.zeros(10, np.float32),
                 hyper=np.zeros(6))
    with pytest.raises(ValueError):
        pkg.LearnedDecimation("cpu").load_checkpoint(path)
