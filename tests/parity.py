"""Comparison of HIP-path outputs with the fp64 oracle.

Tolerances (the reading of "float stages within 1e-5 relative" and "mask
bit-exact except within 1e-4 of the threshold" used throughout):

* float stages B, L, G: |gpu - ora| <= 1e-5 * max(|ora|, max|ORA|) per pixel
  (a relative bound with a normwise floor: pure elementwise relative error
  is not attainable where a stage crosses zero);
* the max M: |M_gpu - M_ora| <= 1e-5 * M_ora;
* mask: bit-exact except (a) band pixels, |G_ora - tau_ora| <= 1e-4, and (b)
  sign-ambiguous pixels, whose 3x3 window holds an L_ora with
  0 < |L_ora| <= 1e-5 * max|L_ora| (where fp32 rounding may flip L's sign).
  Both kinds are counted and reported, and the differing ones are bounded
  (exempt_bounded); Z may differ only at (b).
"""
import numpy as np
import scipy.ndimage as ndi

REL = 1e-5
BAND = 1e-4


def float_stage_ok(gpu, ora):
    gpu = np.asarray(gpu, np.float64)
    bound = REL * np.maximum(np.abs(ora), np.max(np.abs(ora)) if ora.size else 0.0)
    err = np.abs(gpu - ora)
    bad = err > bound
    return int(bad.sum()), float(err.max()) if err.size else 0.0


def exemptions(ora, theta):
    """Boolean maps (band, ambiguous) from the oracle's stage outputs."""
    tau = theta * ora["M"]
    band = np.abs(ora["G"] - tau) <= BAND
    L = ora["L"]
    lmax = np.max(np.abs(L)) if L.size else 0.0
    tiny = (np.abs(L) <= REL * lmax) & (L != 0)
    amb = ndi.maximum_filter(tiny, 3, mode="nearest") if L.size else tiny
    return band, amb


def compare_mask(mask, ora, theta):
    """Returns dict(mismatch=#unexempt mismatches, band=#band, amb=#ambiguous,
    exempt_diff=#differing exempt pixels, band_diff / amb_diff = those in
    each kind)."""
    band, amb = exemptions(ora, theta)
    ex = band | amb
    diff = np.asarray(mask) != ora["mask"]
    return dict(mismatch=int((diff & ~ex).sum()), band=int(band.sum()),
                amb=int(amb.sum()), exempt_diff=int((diff & ex).sum()),
                band_diff=int((diff & band).sum()), amb_diff=int((diff & amb).sum()))


# Exempt pixels may differ (fp32 against fp64), but only as rare flips: at
# most 1% of each kind, plus 2.  An fp32 G is within about 1e-6 relative of
# the oracle's, so only band pixels that close to tau can flip, a small
# fraction of a band 1e-4 wide; likewise for the signs of near-zero L.
EXEMPT_FRAC = 0.01
EXEMPT_SLACK = 2


def exempt_bounded(r):
    """True when the differing exempt pixels of compare_mask's result r (or a
    sum of such results) are within the bound above."""
    return (r["band_diff"] <= EXEMPT_FRAC * r["band"] + EXEMPT_SLACK and
            r["amb_diff"] <= EXEMPT_FRAC * r["amb"] + EXEMPT_SLACK)


def compare_stages(st, ora, theta):
    """st: numpy dict with B, L, G, Z, M, mask from the stage hook."""
    out = {}
    for k in ("B", "L", "G"):
        out[k] = float_stage_ok(st[k], ora[k])
    M = float(st["M"])
    out["M_ok"] = abs(M - ora["M"]) <= REL * ora["M"] if ora["M"] > 0 else M == 0.0
    band, amb = exemptions(ora, theta)
    out["Z_mismatch"] = int(((st["Z"] != ora["Z"]) & ~amb).sum())
    out["mask"] = compare_mask(st["mask"], ora, theta)
    return out
