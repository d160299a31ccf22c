"""Error measures shared by the parity tests (no method arithmetic here).

Bar: GPU-FP64 within 1e-12 relative and FP32 within 1e-4 relative, per
voxel, over voxels above 1e-6 of their group's largest |fluence|.

Pure diamond difference (fixup off) can give negative scalar fluence.  At a
voxel whose fluence differs in sign from a face neighbour's, the value is a
small difference of large terms, and the relative error is ill-conditioned:
a random one-ulp change of every cross section and density moves the
oracle's own result there by up to ~1e-12 in S2, 10 to 30 times more than
elsewhere (pinned in test_oracle_conditioning.py).  Only those voxels are measured against
their group's largest |fluence| instead of their own value.
"""
import numpy as np


def sign_change_voxels(phi_g, shape):
    """Mask [V] of the voxels whose fluence has another sign than at least
    one face neighbour (shape = (nx, ny, nz), v = i + nx (j + ny k))."""
    nx, ny, nz = shape
    a = np.sign(np.asarray(phi_g).reshape(nz, ny, nx))
    m = np.zeros(a.shape, bool)
    for ax in range(3):
        d = np.diff(a, axis=ax) != 0
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        m[tuple(lo)] |= d
        m[tuple(hi)] |= d
    return m.reshape(-1)


def rel_err(got, want, floor=1e-6):
    """Largest |got - want| / |want| over voxels above `floor` of their
    group's largest |want| (arrays [G][V])."""
    got = np.asarray(got).reshape(want.shape)
    worst = 0.0
    for g in range(want.shape[0]):
        m = np.abs(want[g]).max()
        if m == 0:
            assert np.abs(got[g]).max() == 0
            continue
        sel = np.abs(want[g]) > floor * m
        worst = max(worst, (np.abs(got[g] - want[g])[sel] / np.abs(want[g][sel])).max())
    return worst


def l2_rel(got, want):
    got = np.asarray(got).reshape(want.shape)
    return np.linalg.norm(got - want) / np.linalg.norm(want)


def parity_err(got, want, prob, l2_bar=1e-13, floor=1e-6):
    """Per-voxel relative error as rel_err, except at voxels next to a sign
    change of the fluence (see the module note), which are measured against
    their group's largest |want|; with any such voxel the global relative L2
    error must also stay under l2_bar."""
    got = np.asarray(got).reshape(want.shape)
    shape = (prob.nx, prob.ny, prob.nz)
    worst, any_sc = 0.0, False
    for g in range(want.shape[0]):
        m = np.abs(want[g]).max()
        if m == 0:
            assert np.abs(got[g]).max() == 0
            continue
        sc = sign_change_voxels(want[g], shape)
        any_sc = any_sc or bool(sc.any())
        sel = (np.abs(want[g]) > floor * m) & ~sc
        err = np.abs(got[g] - want[g])
        if sel.any():
            worst = max(worst, (err[sel] / np.abs(want[g][sel])).max())
        if sc.any():
            worst = max(worst, err[sc].max() / m)
    if any_sc:
        assert l2_rel(got, want) < l2_bar
    return worst


def sampled_rel_err(got, golden, floor=1e-6):
    """Largest relative error of a full GPU result got [G][V] against a
    stored golden (sampled voxels idx, values phi [G][K], group maxima gmax
    [G]) over the sampled voxels above `floor` of their group's maximum.
    Returns (error, number of voxels compared)."""
    got = np.asarray(got)
    idx, phi, gmax = golden["idx"], golden["phi"], golden["gmax"]
    worst, n = 0.0, 0
    for g in range(phi.shape[0]):
        if gmax[g] == 0:
            continue
        sel = np.abs(phi[g]) > floor * gmax[g]
        e = np.abs(got[g][idx][sel] - phi[g][sel]) / np.abs(phi[g][sel])
        if e.size:
            worst = max(worst, float(e.max()))
        n += int(sel.sum())
    return worst, n
