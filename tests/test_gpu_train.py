"""The trainer end to end on a few generated pairs: interrupted and resumed
from its checkpoint, it reaches bit for bit the state of an uninterrupted
run (data regenerated from the seeds, permutation from seed and epoch,
ordered weight-gradient reduction)."""
import argparse

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _args(tmp, **kw):
    a = dict(pairs=32, first_seed=500, epochs=2, batch=16, lr=2e-3, seed=3, checkpoint="", save_every=1,
             resume=False, stop_after=0, log_every=1, out="")
    a.update(kw)
    return argparse.Namespace(**a)


def test_trainer_resume_matches_uninterrupted(tmp_path):
    import torch
    from paper_2012_10802_amd import train_window as T
    logs = []
    straight = T.train(_args(tmp_path, out=str(tmp_path / "a.npz")), log=logs.append)
    ck = str(tmp_path / "ck.npz")
    T.train(_args(tmp_path, checkpoint=ck, stop_after=2), log=logs.append)
    resumed = T.train(_args(tmp_path, checkpoint=ck, resume=True, out=str(tmp_path / "b.npz")), log=logs.append)
    torch.cuda.synchronize()
    assert straight.step == resumed.step == 4
    for name in ("params", "m", "v"):
        np.testing.assert_array_equal(getattr(straight, name).cpu().numpy(), getattr(resumed, name).cpu().numpy(),
                                      err_msg=name)
    assert any("resumed at step 2" in m for m in logs)
