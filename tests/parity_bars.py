"""Parity bars of the GNN against the FP64 oracle -- test-side only.

Forward (the predicted factor L).  Only part of L is network output: in
diag_mode 1 the diagonal is sqrt(A_ii) and carries no network term, and in
every mode it dominates ||L||, so a norm over all entries would hide errors
in the entries the network actually predicts.  The bars therefore split L:

  * strictly lower entries (the decoded pair averages): relative Frobenius
    <= OFF_REL and, entry by entry, |L - L_ref| <= ELEM * (|L_ref| + rms),
    rms = root mean square of the reference's strictly lower entries.  The
    element-wise form catches a localised error (values stored in the wrong
    columns of some rows) that a norm over a million entries would absorb;
  * diagonal, modes 0 and 2 (network output through a softplus): the same
    two bars on the diagonal entries;
  * diagonal, mode 1 (sqrt(A_ii), no network term): within two FP32 ulps.

Calibration: tests/bf16_emul.py replays the network with every BF16
rounding the GPU makes (its error on the shipped network's 12^3 smoke
system, 2.3e-3 relative over all entries, matches the GPU's 2.0e-3).  Its
distance to the oracle is at most 8.8e-3 relative Frobenius on the strictly
lower part and 1.2e-2 element-wise in the above form (random weights:
1e-3 / 1.5e-3 at h = 32, 4e-3 / 5.4e-3 at h = 64 with 5 layers; the worst
case is a shipped trained network), so the bars leave a factor of 2.3-2.5
over the worst case and about 5 over random weights.

Reverse mode (parameter gradients).  Per tensor, the GPU's relative error
and 1 - cosine must stay within GRAD_FACTOR times the BF16 emulation's on
the same inputs (floors GRAD_REL_FLOOR and GRAD_COS_FLOOR), and the whole
flattened gradient keeps cosine >= 0.999 and relative error <= 0.05.  The
emulation sets the scale per tensor: the encoders' [1 x h] weight gradients
sum n signed terms and lose digits to cancellation (relative error up to
0.4 at h = 64 with 5 layers), while a tensor such as dec.b1 is accurate to
1e-3, so a fixed bar would be either loose for one or flaky for the other.
A tensor scaled by 2 (relative error 1) fails the per-tensor bar."""
from __future__ import annotations

import numpy as np

OFF_REL = 2e-2
ELEM = 3e-2
GRAD_FACTOR = 6.0
GRAD_REL_FLOOR = 0.05
GRAD_COS_FLOOR = 0.01
U32 = 2.0 ** -24


def lower_masks(pat):
    row = np.repeat(np.arange(pat.n), np.diff(pat.lrowptr))
    diag = pat.lcol == row
    return diag, ~diag


def _part(lg, ref, mask, what):
    if not mask.any():
        return {f"{what}_rel": 0.0, f"{what}_elem": 0.0}
    a, r = lg[mask], ref[mask]
    nr = np.linalg.norm(r)
    rms = np.sqrt(np.mean(r * r))
    rel = np.linalg.norm(a - r) / nr if nr > 0 else np.linalg.norm(a - r)
    elem = np.abs(a - r) / (np.abs(r) + (rms if rms > 0 else 1.0))
    k = int(np.argmax(elem))
    assert rel <= OFF_REL, f"{what}: relative Frobenius {rel:.3e} > {OFF_REL}"
    assert elem[k] <= ELEM, (f"{what}: entry {np.flatnonzero(mask)[k]} differs by {elem[k]:.3e} "
                             f"of (|ref| + rms) > {ELEM} (gpu {a[k]!r}, ref {r[k]!r})")
    return {f"{what}_rel": float(rel), f"{what}_elem": float(elem[k])}


def check_factor(pat, lg, ref, diag_mode):
    """Assert the forward bars on L (lower CSR order) and return the stats."""
    lg, ref = np.asarray(lg, np.float64), np.asarray(ref, np.float64)
    diag, off = lower_masks(pat)
    assert np.all(np.isfinite(lg)), "non-finite factor entries"
    assert np.all(lg[diag] > 0), "non-positive diagonal"
    st = _part(lg, ref, off, "off")
    if diag_mode == 1:
        err = np.abs(lg[diag] - ref[diag])
        assert np.all(err <= 2 * U32 * np.abs(ref[diag])), \
            f"diagonal sqrt(A_ii): max rel {np.max(err / ref[diag]):.3e}"
        st["diag_rel"] = float(np.max(err / ref[diag]))
    else:
        st.update(_part(lg, ref, diag, "diag"))
    return st


def check_vector(v, ref, what="x0"):
    """The forward bars for a node-level network output (the x^0 head)."""
    v, ref = np.asarray(v, np.float64), np.asarray(ref, np.float64)
    assert np.all(np.isfinite(v))
    return _part(v, ref, np.ones(v.shape[0], bool), what)


def _cos(a, r):
    na, nr = np.linalg.norm(a), np.linalg.norm(r)
    return float(a @ r / (na * nr)) if na > 0 and nr > 0 else (1.0 if na == nr else 0.0)


def check_grads(G, R, Em, keys):
    """G: GPU gradient, R: FP64 oracle, Em: BF16 emulation; dicts of arrays
    over `keys`.  Asserts the reverse-mode bars; returns the worst tensor."""
    fa = np.concatenate([np.asarray(G[k], np.float64).ravel() for k in keys])
    fr = np.concatenate([np.asarray(R[k], np.float64).ravel() for k in keys])
    cos_all = _cos(fa, fr)
    rel_all = np.linalg.norm(fa - fr) / np.linalg.norm(fr)
    assert cos_all >= 0.999 and rel_all <= 0.05, ("whole gradient", cos_all, rel_all)
    worst = (0.0, "")
    for k in keys:
        a = np.asarray(G[k], np.float64).ravel()
        r = np.asarray(R[k], np.float64).ravel()
        e = np.asarray(Em[k], np.float64).ravel()
        nr = np.linalg.norm(r)
        if nr == 0:
            assert np.linalg.norm(a) <= 1e-6, (k, "gradient should be zero")
            continue
        rel, rel_e = np.linalg.norm(a - r) / nr, np.linalg.norm(e - r) / nr
        dc, dc_e = 1.0 - _cos(a, r), 1.0 - _cos(e, r)
        bar_rel = max(GRAD_FACTOR * rel_e, GRAD_REL_FLOOR)
        bar_cos = max(GRAD_FACTOR * dc_e, GRAD_COS_FLOOR)
        assert rel <= bar_rel, f"{k}: relative error {rel:.3e} > {bar_rel:.3e} (BF16 model {rel_e:.3e})"
        assert dc <= bar_cos, f"{k}: 1 - cosine {dc:.3e} > {bar_cos:.3e} (BF16 model {dc_e:.3e})"
        if rel / bar_rel > worst[0]:
            worst = (rel / bar_rel, k)
    return {"cos_all": cos_all, "rel_all": float(rel_all), "worst_fraction_of_bar": worst}
