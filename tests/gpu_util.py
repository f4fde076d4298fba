"""Helpers for the GPU tests: move seeded numpy inputs to the device, run the
library through its C ABI binding, and measure errors against the oracle."""
import numpy as np


def torch_mod():
    import torch
    return torch


def to_dev(a: np.ndarray, dtype: str):
    torch = torch_mod()
    td = torch.float32 if dtype == "f32" else torch.float64
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0", dtype=td)


def rounded_input(a: np.ndarray, dtype: str) -> np.ndarray:
    """The exact values the GPU sees: float32 rounding for f32, unchanged for f64."""
    return a.astype(np.float32).astype(np.float64) if dtype == "f32" else a.astype(np.float64)


def gpu_periodic(a: np.ndarray, coeffs, T: int, dtype: str) -> np.ndarray:
    import paper_2105_06676_amd as sfft
    torch = torch_mod()
    g = to_dev(a, dtype)
    sfft.periodic(g, coeffs, T)
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64)


def gpu_aperiodic(a: np.ndarray, coeffs, T: int, dtype: str) -> np.ndarray:
    import paper_2105_06676_amd as sfft
    torch = torch_mod()
    g = to_dev(a, dtype)
    sfft.aperiodic(g, coeffs, T)
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64)


def rel_l2(y: np.ndarray, ref: np.ndarray) -> float:
    den = np.linalg.norm(ref)
    num = np.linalg.norm(y - ref)
    return float(num / den) if den > 0 else float(num)


def max_abs_rel(y: np.ndarray, ref: np.ndarray) -> float:
    """max |y - ref| / max |ref|: the largest single-cell error on the scale of the result."""
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    num = float(np.max(np.abs(y - ref))) if ref.size else 0.0
    return num / den if den > 0 else num


def errors(y: np.ndarray, ref: np.ndarray) -> dict:
    return {"rel_l2": rel_l2(y, ref), "max_abs": float(np.max(np.abs(y - ref))) if ref.size else 0.0,
            "max_abs_rel": max_abs_rel(y, ref)}


def assert_close(y: np.ndarray, ref: np.ndarray, tol: float, what=None) -> None:
    """Both gates: relative L2 error and the largest cell error relative to max |ref|
    are each at most tol (a norm alone would hide a few bad cells in a large grid)."""
    assert y.shape == ref.shape, (y.shape, ref.shape, what)
    assert np.all(np.isfinite(y)), ("non-finite output", what)
    e = errors(y, ref)
    assert e["rel_l2"] <= tol and e["max_abs_rel"] <= tol, (e, tol, what)


# Tolerances stated for the path against the FP64 oracle (relative L2 and the
# largest cell error relative to max |ref|).
TOL = {"f32": 1e-5, "f64": 1e-12}
