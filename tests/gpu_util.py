"""Helpers shared by the GPU parity tests (inputs only; no method arithmetic)."""
import numpy as np
import torch

from paper_2311_15038_amd import synth


def dev():
    return torch.device("cuda:0")


def to_dev_u16(a: np.ndarray) -> torch.Tensor:
    return synth.from_numpy_u16(a, dev())


def u16_np(t: torch.Tensor) -> np.ndarray:
    return synth.to_numpy_u16(t)


def u64_np(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def u32_np(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def hist_to_dev(h: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(h, dtype=np.uint64).view(np.int64)).to(dev())


def bits_to_dev(b: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(b, dtype=np.uint32).view(np.int32)).to(dev())


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
