"""Helpers shared by the GPU parity tests: build the same seeded workload for the
HIP library (through the binding) and for the CPU oracle."""
import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().to("cpu").to(torch.float64).numpy()


def relerr(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def colwise_relerr(a, b):
    a = np.asarray(a).reshape(-1, np.asarray(a).shape[-1])
    b = np.asarray(b).reshape(-1, np.asarray(b).shape[-1])
    return float(np.max(np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), 1e-300)))


class Pair:
    """A workload instantiated on both sides: `orc` (oracle Problem) and
    `gpu` (rp4d.Problem) with identical x_b and y, plus the GPU trajectory at x_b."""

    def __init__(self, cfg, seed=0, ckpt_every=0, ctx=None):
        from oracle.problem import make_problem
        from paper_2401_15758_amd import inputs, rp4d
        self.cfg = cfg
        self.orc = make_problem(cfg, inputs.draws(cfg, seed=seed))
        self.ctx = ctx or rp4d.Context(0)
        self.gpu = rp4d.Problem(self.ctx, cfg, ckpt_every=ckpt_every)
        self.gpu.set_data(to_dev(self.orc.xb), to_dev(self.orc.y.reshape(-1)))
        self.traj = self.gpu.traj()
        self.xb_dev = to_dev(self.orc.xb)
        self.Jobs = self.gpu.fwd(self.xb_dev, self.traj)
        self._otraj = None

    @property
    def otraj(self):
        if self._otraj is None:
            self._otraj = self.orc.fwd(self.orc.xb)
        return self._otraj
