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
    """The parity_err measure of a full GPU result got [G][V] against a
    stored golden (sampled voxels idx, values phi [G][K], group maxima gmax
    [G], sign-change flags sc [G][K]) over the sampled voxels: per voxel
    relative above `floor` of the group maximum, flagged voxels against the
    group maximum.  Returns (error, voxels compared, error over the flagged
    voxels alone)."""
    got = np.asarray(got)
    idx, phi, gmax, sc = golden["idx"], golden["phi"], golden["gmax"], golden["sc"]
    worst, worst_sc, n = 0.0, 0.0, 0
    for g in range(phi.shape[0]):
        if gmax[g] == 0:
            continue
        err = np.abs(got[g][idx] - phi[g])
        sel = (np.abs(phi[g]) > floor * gmax[g]) & ~sc[g]
        if sel.any():
            worst = max(worst, float((err[sel] / np.abs(phi[g][sel])).max()))
        if sc[g].any():
            worst_sc = max(worst_sc, float(err[sc[g]].max() / gmax[g]))
        n += int(sel.sum() + sc[g].sum())
    return max(worst, worst_sc), n, worst_sc


def sampled_fp32_excess(got, golden, floor=1e-6, bar=1e-4, factor=4.0):
    """FP32 parity against a stored golden, as a ratio that must stay below
    1: at every sampled voxel above `floor` of its group's maximum, the error
    over the larger of `bar` times the voxel's value and, where the golden
    holds the single-precision model of a pure diamond-difference solve
    (phi_single), `factor` times that model's own deviation from the double
    solution (in optically thick pure-DD groups the outflow 2 psi - psi_in
    cancels, and single-precision cells alone move low-fluence voxels by
    more than 1e-4 there).  Voxels next to a sign change are measured against
    the group maximum as in sampled_rel_err.  Returns (ratio, voxels
    compared, voxels where the single-precision allowance was the larger)."""
    got = np.asarray(got)
    idx, phi, gmax, sc = golden["idx"], golden["phi"], golden["gmax"], golden["sc"]
    single = golden["phi_single"] if "phi_single" in golden else None
    worst, n, n_wide = 0.0, 0, 0
    for g in range(phi.shape[0]):
        if gmax[g] == 0:
            continue
        err = np.abs(got[g][idx] - phi[g])
        sel = (np.abs(phi[g]) > floor * gmax[g]) & ~sc[g]
        allow = bar * np.abs(phi[g])
        if single is not None:
            wide = factor * np.abs(single[g] - phi[g])
            n_wide += int((sel & (wide > allow)).sum())
            allow = np.maximum(allow, wide)
        if sel.any():
            worst = max(worst, float((err[sel] / allow[sel]).max()))
        if sc[g].any():
            worst = max(worst, float(err[sc[g]].max() / gmax[g] / bar))
        n += int(sel.sum() + sc[g].sum())
    return worst, n, n_wide
