"""Device-buffer helpers for the GPU tests (torch is only memory and streams)."""
import numpy as np
import torch


def dev():
    return torch.device("cuda:0")


def to_device(a: np.ndarray) -> torch.Tensor:
    """Bytes of a host array in a fresh (256-byte aligned) device buffer."""
    return torch.from_numpy(np.ascontiguousarray(a).view(np.uint8).reshape(-1)).to(dev())


def empty_like_bytes(a: np.ndarray) -> torch.Tensor:
    return torch.empty(a.nbytes, dtype=torch.uint8, device=dev())


def to_host(t: torch.Tensor, like: np.ndarray) -> np.ndarray:
    return t.cpu().numpy().view(like.dtype).reshape(like.shape)


def stream():
    return torch.cuda.current_stream()


def sync():
    torch.cuda.synchronize()
