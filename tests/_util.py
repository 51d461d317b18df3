"""Helpers shared by the GPU tests: layout conversion and oracle/GPU setup of
the same canonical float32 inputs."""
import numpy as np

from paper_2603_00839_amd import synth
from oracle.operator import Operator, make_observation
from oracle.sketch import Sketch


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(synth.to_device_layout(np.asarray(x, np.float32))).cuda()
    return t if dtype is None else t.to(dtype)


def from_dev(t):
    return synth.from_device_layout(t.float().cpu().numpy()).astype(np.float64)


def bf16_round(a):
    """float32 -> nearest bfloat16 (ties to even) -> float64, on the host."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def oracle_pair(p):
    return Operator(p.a1_band, p.a2_band, p.b_band), Sketch(p.om1, p.om2, p.om3)


def gpu_pair(p):
    from paper_2603_00839_amd import rtg
    I1, I2, J = p.dims
    return (rtg.setup_operator(I1, I2, J, p.a1_band, p.a2_band, p.b_band),
            rtg.setup_sketch(I1, I2, J, p.om1, p.om2, p.om3))


def observation(p):
    """Canonical float32 observation C and the noise norm delta (oracle)."""
    op, _ = oracle_pair(p)
    C, delta, _ = make_observation(op, p.x_true, p.noise_dir, p.nu)
    return C.astype(np.float32), float(delta)


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def maxrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
