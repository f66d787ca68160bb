"""Parity of compositing outputs where a float32 decision may legitimately
differ from the float64 one.

Every pixel is checked.  A pixel whose kernel output does not match the
oracle's walk (Eq. 3, Algorithm 1) is walked again with its near decisions
(a skip of a positive exponent, a skip below alpha = 1/255, the
transmittance stop; near = within 1e-5 of the threshold, relative, the
stop's distance divided by the transmittance's condition number) taken the
other way, in every combination of up to MAX_NEAR of them.  It passes if
the kernel matches one of these outcomes at the same tolerance.  Pixels
that match none are counted and may be at most 0.1 % of the pixels checked.
"""
from __future__ import annotations

import numpy as np

THR = 1e-5            # nearness of a decision to its threshold (relative)
MAX_NEAR = 8          # combinations of up to this many near decisions are tried
UNMATCHED_FRAC = 1e-3


def check_flips(orc, cam, ranges, ids, mean2d, conic, opacity, topk_idx, topk_w, L, pix, close, base=None,
                label=""):
    """pix: flat pixel indices (npix,).  close(sel, coef, fT, last) -> bool
    array over sel: whether the kernel's outputs of pixels pix[sel] match the
    given oracle outcome (coef [len(sel), levels, L], final_T, last).  base:
    the plain walk of every pixel of pix (coef [npix, levels, L], final_T,
    last) if already computed.  Returns a dict of counts, the indices (into
    pix) of the unmatched pixels, the mask of pixels that match the plain walk
    (base_ok) and that walk (base); asserts the 0.1 % bar."""
    args = (cam, ranges, ids, mean2d, conic, opacity, topk_idx, topk_w, L)
    pix = np.asarray(pix, np.int64)
    npix = pix.shape[0]
    if base is None:
        coef, fT, last, _ = orc.composite_pixels_alt(*args, pix, 0, THR)
    else:
        coef, fT, last = base
    ok = np.asarray(close(np.arange(npix), coef, fT, last), bool)
    bad = np.nonzero(~ok)[0]
    matched = np.zeros(bad.shape[0], bool)
    if bad.size:
        _, _, _, nn = orc.composite_pixels_alt(*args, pix[bad], 0, THR)
        nn = np.minimum(nn.astype(np.int64), MAX_NEAR)
        for mask in range(1, 1 << MAX_NEAR):
            need = mask.bit_length()
            open_ = ~matched
            if not open_.any() or need > nn[open_].max():
                break
            sel = np.nonzero(open_ & (nn >= need))[0]
            if sel.size == 0:
                continue
            c2, t2, l2, n2 = orc.composite_pixels_alt(*args, pix[bad[sel]], mask, THR)
            nn[sel] = np.maximum(nn[sel], np.minimum(n2, MAX_NEAR))
            matched[sel] |= np.asarray(close(bad[sel], c2, t2, l2), bool)
    unmatched = bad[~matched]
    res = dict(checked=npix, base_mismatch=int(bad.size), matched_flip=int(matched.sum()),
               unmatched=int(unmatched.size), unmatched_idx=unmatched, base_ok=ok, base=(coef, fT, last))
    print("%s%d pixels checked: %d match the oracle walk, %d match it with near decisions flipped, %d match neither"
          % (label + ": " if label else "", npix, npix - bad.size, res["matched_flip"], res["unmatched"]))
    assert unmatched.size <= UNMATCHED_FRAC * npix, (
        "%d of %d pixels match no outcome of the oracle walk (bar %.1f %%)" % (unmatched.size, npix,
                                                                            100 * UNMATCHED_FRAC))
    return res


def coef_close(got_coef, got_T, got_last, atol):
    """close() for coefficient maps: got_coef [npix, levels, L], got_T and
    got_last [npix] (the kernel's values of the checked pixels, in pix
    order); max abs error over levels and atoms and of T within atol, last
    equal."""
    def close(sel, coef, fT, last):
        e = np.abs(got_coef[sel] - coef).reshape(len(sel), -1).max(axis=1) if len(sel) else np.zeros(0)
        return (e <= atol) & (np.abs(got_T[sel] - fT) <= atol) & (got_last[sel] == last)
    return close
