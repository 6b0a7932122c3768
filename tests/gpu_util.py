"""Helpers for the GPU tests: host <-> device column-major transfers and error measures."""
import numpy as np
import torch

EPS = 2.0 ** -52


def to_dev(A: np.ndarray, ld: int | None = None) -> torch.Tensor:
    """Column-major float64 device copy of a 2-D numpy array (optionally padded to ld rows)."""
    A = np.asarray(A, dtype=np.float64)
    q, r = A.shape
    ld = q if ld is None else ld
    base = torch.zeros((r, ld), dtype=torch.float64)
    base[:, :q] = torch.from_numpy(np.ascontiguousarray(A.T))
    return base.cuda().t()[:q, :]


def to_host(T: torch.Tensor) -> np.ndarray:
    return np.asfortranarray(T.t().cpu().numpy().T)


def recon_ratio(Y, Q, R):
    return np.linalg.norm(Y - Q @ R) / (Y.shape[0] * EPS * np.linalg.norm(Y))


def orth_ratio(Q):
    return np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])) / (Q.shape[0] * EPS)


def hpl_ratio(Y, x, b):
    n = Y.shape[0]
    return np.abs(Y @ x - b).max() / (np.abs(Y).sum(axis=1).max() * np.abs(x).max() * n * EPS)
