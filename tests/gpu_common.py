"""Helpers shared by the GPU parity tests: run the HIP path on seeded inputs and bring results
back as numpy arrays for comparison with the oracle."""
import numpy as np
import pytest
import torch

from paper_2506_12727_amd import scenes
from paper_2506_12727_amd.raster import GaussianTensors, Rasterizer

# tolerances (images: 1e-5 relative + 1e-6 absolute; gradients: 1e-3 relative)
IMG_RTOL, IMG_ATOL = 1e-5, 1e-6
GRAD_RTOL, GRAD_INF = 1e-3, 1e-4
GRAD_L2 = 1e-3
# at most this fraction of pixels may be flagged (a decision within the kernel's error of its threshold)
FLAG_MAX = 1e-3


def needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run_forward(scene, cams, tile=(16, 16), rast=None, ppl=0):
    r = rast or Rasterizer(tile, ppl)
    g = GaussianTensors.from_scene(scene)
    imgs, fr = r.forward(g, cams)
    torch.cuda.synchronize()
    return r, g, imgs, fr


def to_np(ts):
    return [t.detach().cpu().numpy().astype(np.float64) for t in ts]


def compare_images(gpu, ora, flags, rtol=IMG_RTOL, atol=IMG_ATOL):
    """Element-wise image check outside flagged pixels; returns the flagged fraction."""
    nflag = ntot = 0
    for a, b, f in zip(gpu, ora, flags):
        ok = f == 0
        nflag += int((~ok).sum())
        ntot += ok.size
        err = np.abs(a - b)
        lim = rtol * np.abs(b) + atol
        bad = (err > lim) & ok[None] if a.ndim == 3 else (err > lim) & ok
        if bad.any():
            idx = np.argwhere(bad)[:5]
            raise AssertionError(f"{int(bad.sum())} elements out of tolerance, e.g. {idx.tolist()}: "
                                 f"gpu {a[tuple(idx[0])]} oracle {b[tuple(idx[0])]}")
    return nflag / max(ntot, 1)


def compare_grad(name, gpu, ora, rtol=GRAD_RTOL, inf=GRAD_INF, l2=GRAD_L2, mask=None, extra=None):
    """extra: an added per-element tolerance (broadcast against the gradient), see cov_tolerance."""
    gpu = np.asarray(gpu, np.float64).reshape(ora.shape)
    if mask is not None:
        gpu, ora = gpu[mask], ora[mask]
    scale = np.abs(ora).max()
    assert scale > 0, f"{name}: oracle gradient is all zero"
    err = np.abs(gpu - ora)
    lim = rtol * np.abs(ora) + inf * scale
    if extra is not None:
        lim = lim + extra
    bad = err > lim
    frac_bad = bad.mean()
    rel_l2 = np.linalg.norm(gpu - ora) / np.linalg.norm(ora)
    assert rel_l2 <= l2, f"{name}: relative L2 error {rel_l2:.3e}"
    assert not bad.any(), (f"{name}: {int(bad.sum())} of {bad.size} elements out of tolerance; worst "
                           f"{err.max():.3e} vs scale {scale:.3e}")
    return rel_l2


def grad_flags(scene, cams, tile=(16, 16)):
    """Per-view flags of the oracle's double-geometry walk (the one its gradients take): pixels where
    a cut, clamp or stop decision lies within the kernel's possible error of its threshold."""
    import oracle
    return oracle.forward(scene, cams, tile, geom32_mode=False)["flags"]


def flag_fraction(flags) -> float:
    n = sum(int((f != 0).sum()) for f in flags)
    return n / max(1, sum(f.size for f in flags))


def zero_flagged(dl, flags):
    """dL/dimage (GPU tensors [3,H,W], in place) set to zero at flagged pixels, so that they
    contribute to neither side of a gradient comparison."""
    for t, f in zip(dl, flags):
        t.mul_(torch.from_numpy((f == 0).astype(np.float32)).to(t.device)[None])
    return dl


# relative accuracy of the kernel's float32 sums of per-pixel gradient terms (the measured relative
# L2 error of the mean and opacity gradients at full size is 3e-6-1e-5)
SUM_REL = 1e-5


def conditioning(geoms) -> np.ndarray:
    """Largest condition number over the given views (oracle.geom32 dicts) of each Gaussian's
    projected 2D covariance (1 where it takes part in none)."""
    kappa = None
    for g in geoms:
        a, b, c = (g[k].astype(np.float64) for k in ("ca", "cb", "cc"))
        half_tr = 0.5 * (a + c)
        disc = np.sqrt(np.maximum(half_tr * half_tr - (a * c - b * b), 0.0))
        k = np.where(g["participates"] == 1, (half_tr + disc) / np.maximum(half_tr - disc, 1e-300), 1.0)
        kappa = k if kappa is None else np.maximum(kappa, k)
    return kappa


def cov_tolerance(ora_rows: np.ndarray, kappa: np.ndarray) -> np.ndarray:
    """Added tolerance for the gradients of the covariance parameters (scales, quats) of a Gaussian
    whose projected covariance has condition number kappa: the kernel sums dL/dconic over pixels in
    image axes, and the part that reaches a needle-shaped Gaussian's thin axis is a difference of
    terms about kappa times larger (the long axis' extent squared), so the float32 sums' relative
    error SUM_REL reaches that row amplified by kappa. Per element: SUM_REL kappa |row|."""
    rows = ora_rows.reshape(ora_rows.shape[0], -1)
    return (SUM_REL * kappa * np.linalg.norm(rows, axis=1))[:, None] * np.ones_like(rows)
