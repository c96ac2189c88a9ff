"""CPU checks of the training checkpoint file: a file of another format
version, or written by a run with other arguments, is refused before any
state is loaded."""
import json

import numpy as np
import pytest
import torch

from paper_2311_09265_amd import proposal


def _write(path, **meta):
    base = {"version": proposal.CHECKPOINT_VERSION, "step": 2, "steps": 10, "batch": 4, "lr": 1e-3, "seed": 3,
            "adam_step": 2}
    base.update(meta)
    z = np.zeros(4, np.float32)
    np.savez(path, params=z, adam_m=z, adam_v=z, rng=torch.Generator().get_state().numpy(),
             meta=np.frombuffer(json.dumps(base).encode(), np.uint8))


def test_other_version_is_refused(tmp_path):
    path = str(tmp_path / "c.npz")
    _write(path, version=proposal.CHECKPOINT_VERSION + 1)
    with pytest.raises(ValueError, match="version"):
        proposal.load_checkpoint(None, path, torch.Generator())


def test_other_run_arguments_are_refused(tmp_path):
    class NoGPU:
        device = "cpu"

        def fb_unet_load_state(self, *a):
            pass
    path = str(tmp_path / "c.npz")
    _write(path, steps=11)
    x = torch.zeros(2, 8, 8, 6)
    with pytest.raises(ValueError, match="other arguments"):
        proposal.train(NoGPU(), x, x[..., :2], x[..., 0], steps=10, batch=4, lr=1e-3, seed=3, ckpt=path, resume=True)
