"""Helpers for the GPU parity tests (host <-> device copies, sentinels)."""
import numpy as np
import torch

DEV = "cuda:0"


def to_dev(a: np.ndarray, pad_before: int = 0, pad_after: int = 0, fill: int = 0xA5) -> torch.Tensor:
    """Copy a uint8 numpy array to the GPU.  With padding, the returned tensor
    is a view that starts ``pad_before`` bytes into a larger buffer (for
    misaligned-pointer tests); the padding holds ``fill``."""
    a = np.ascontiguousarray(a, dtype=np.uint8).reshape(-1)
    if not pad_before and not pad_after:
        return torch.from_numpy(a.copy()).to(DEV)
    big = torch.full((pad_before + a.size + pad_after,), fill, dtype=torch.uint8, device=DEV)
    view = big[pad_before:pad_before + a.size]
    if a.size:
        view.copy_(torch.from_numpy(a.copy()))
    return view


def empty_dev(n: int, pad_before: int = 0, fill: int = 0x3C) -> torch.Tensor:
    big = torch.full((pad_before + n + 16,), fill, dtype=torch.uint8, device=DEV)
    return big[pad_before:pad_before + n]


def to_host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().reshape(-1)


def assert_bytes_equal(got: np.ndarray, want: np.ndarray, what: str):
    got = np.asarray(got).reshape(-1)
    want = np.asarray(want).reshape(-1)
    assert got.size == want.size, "%s: size %d != %d" % (what, got.size, want.size)
    bad = np.nonzero(got != want)[0]
    if bad.size:
        i = int(bad[0])
        raise AssertionError("%s: %d bytes differ, first at %d: got %02x want %02x"
                             % (what, bad.size, i, got[i], want[i]))
