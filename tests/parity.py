"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare it with the oracle on identical inputs.

Tolerance (the parity bar of the FP64 path): per field,
|gpu - oracle| <= 1e-12 * max_over_the_field |oracle|, outside the cutoff
band.  Smoothness flags are bit-identical outside the band.  A face is "in
the band" when the oracle finds some chi_k with |chi_k / C_T - 1| <= 1e-10
on the same input: there the cutoff decision is a matter of round-off, so
the face (and, after a step, its dependency cone) is excluded and counted.
"""
import numpy as np

RTOL = 1e-12


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a GPU")
    import paper_2010_13289_amd as T
    T.lib()  # raises if the HIP library is missing: no fallback path
    return torch


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def field_scale(o):
    """max |o| per field (leading axis), never below the smallest normal."""
    o = np.asarray(o)
    s = np.abs(o.reshape(o.shape[0], -1)).max(axis=1)
    return np.maximum(s, 1e-300)


def assert_close_fields(g, o, exclude=None, rtol=RTOL, what=""):
    """Per-field scaled comparison; exclude: boolean mask broadcastable to
    one field (True = skip).  Returns the largest scaled error."""
    g = np.asarray(g)
    o = np.asarray(o)
    assert g.shape == o.shape, (g.shape, o.shape)
    assert np.all(np.isfinite(g)), f"{what}: non-finite GPU values"
    scale = field_scale(o)
    err = np.abs(g - o) / scale.reshape((-1,) + (1,) * (o.ndim - 1))
    if exclude is not None:
        err = np.where(exclude[None], 0.0, err)
    worst = float(err.max()) if err.size else 0.0
    if worst > rtol:
        idx = np.unravel_index(int(np.argmax(err)), err.shape)
        raise AssertionError(f"{what}: scaled error {worst:.3e} > {rtol:.0e} at {idx}: "
                             f"gpu={g[idx]!r} oracle={o[idx]!r}")
    return worst


def ulp_perturbed(U, seed=97):
    """U with every value moved by -1, 0 or +1 units in the last place."""
    rng = np.random.default_rng(seed)
    return U * (1.0 + np.ldexp(1.0, -52) * rng.choice([-1.0, 0.0, 1.0], size=U.shape))


def one_ulp_spread(o, o_pert, keep=None):
    """Per field, how far the oracle's own output moves when its input moves
    by one ulp (on the kept samples): a diagnostic of the conditioning,
    printed beside the parity error."""
    d = np.abs(np.asarray(o_pert) - np.asarray(o))
    if keep is not None:
        d = d[keep]
    return d.max(axis=0) if d.size else np.zeros(d.shape[-1])


def conditioning_tol(o, o_pert, scale, rtol=RTOL, factor=4.0, keep=None):
    """Per-field tolerance for a multi-step rollout, whose FP64 conditioning
    is worse than one step's: max(rtol * scale, factor * spread), with the
    spread of one_ulp_spread.  Per-call and per-step checks use rtol alone."""
    return np.maximum(rtol * scale, factor * one_ulp_spread(o, o_pert, keep)), one_ulp_spread(o, o_pert, keep)


def band_faces(band):
    """[2][nf][faces...] band bits -> boolean mask over faces."""
    return np.any(band.reshape((-1,) + band.shape[2:]) != 0, axis=0)


def faces_to_cells(face_mask, axis_np, n_axis, periodic, reach):
    """Cells within `reach` cells of a masked face along numpy axis axis_np
    (face j lies between cells j-1 and j)."""
    shape = list(face_mask.shape)
    shape[axis_np] = n_axis
    out = np.zeros(shape, dtype=bool)
    fidx = np.nonzero(face_mask)
    for pos in zip(*fidx):
        j = pos[axis_np]
        for c in range(j - reach, j + reach):
            cc = c % n_axis if periodic else min(max(c, 0), n_axis - 1)
            p = list(pos)
            p[axis_np] = cc
            out[tuple(p)] = True
    return out
