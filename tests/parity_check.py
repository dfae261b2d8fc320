"""Parity verdict between the GPU library and the FP64 oracle (shared by the GPU tests).

Hit ids: bit-exact for every (initial beam, generation) whose path is not flagged by
the oracle up to that generation.  Flags: wherever both sides traced the same segment
(the oracle's path is unflagged before it), the GPU flags it exactly when the oracle
does, so a GPU that flags too much or too little fails.  Per-generation counts: equal
within the number of oracle-flagged beams of earlier generations, and the flagged counts
equal when no flagged path took a different hit.

Microphones: a microphone is strict when the oracle put no energy in its flag channel
(the oracle alone decides).  On strict microphones the GPU's flag energy must be zero,
unless some flagged path took a different hit on the two sides (then its children may
reach other microphones, which the contract allows; such microphones are counted and
held to the non-strict bound).  Strict microphones agree within 0.01 dB (energies above
1e-12 of the maximum) and their summed energy within 1e-4 relative; the others satisfy
|E_gpu - E_orc| <= 2.3e-3 E_orc + E_flag_gpu + E_flag_orc.
"""
from __future__ import annotations

import numpy as np

DB_TOL = 0.01
REL_SUM_TOL = 1e-4
NONSTRICT_REL = 2.3e-3   # 0.01 dB as an energy ratio, rounded up
NOT_TRACED = -2          # hit-array value of a generation a path never reached


def unflagged_mask(flag):
    """True where the oracle path is unflagged up to and including that generation."""
    return np.maximum.accumulate(flag.astype(np.uint8), axis=1) == 0


def unflagged_before(flag):
    """True where the oracle path is unflagged in every generation before that one (the
    GPU then traced the very same segment)."""
    m = unflagged_mask(flag)
    out = np.ones_like(m)
    out[:, 1:] = m[:, :-1]
    return out


def check_hits(orc_hit, orc_flag, orc_t, gpu_hit, gpu_t=None, rows=None):
    if rows is not None:
        gpu_hit = gpu_hit[rows]
        gpu_t = None if gpu_t is None else gpu_t[rows]
    mask = unflagged_mask(orc_flag)
    bad = mask & (orc_hit != gpu_hit)
    n_bad = int(bad.sum())
    assert n_bad == 0, f"{n_bad} unflagged hit mismatches, first at {np.argwhere(bad)[:5].tolist()}: " \
                       f"oracle {orc_hit[bad][:5].tolist()} gpu {gpu_hit[bad][:5].tolist()}"
    if gpu_t is not None:
        m = mask & (orc_hit >= 0)
        dt = np.abs(gpu_t[m] - orc_t[m])
        assert (dt <= 1e-9 * np.maximum(1.0, orc_t[m])).all(), f"max |dt| {dt.max()}"
    return int(mask.sum())


def check_flags(orc_hit, orc_flag, gpu_flag, rows=None):
    """Every segment both sides traced alike carries the same flag.  Returns how many
    segments were compared."""
    if rows is not None:
        gpu_flag = gpu_flag[rows]
    same = unflagged_before(orc_flag) & (orc_hit != NOT_TRACED)
    bad = same & (orc_flag.astype(bool) != gpu_flag.astype(bool))
    n_bad = int(bad.sum())
    over = int((bad & gpu_flag.astype(bool)).sum())
    assert n_bad == 0, f"{n_bad} flag mismatches ({over} flagged by the GPU only), first at " \
                       f"{np.argwhere(bad)[:5].tolist()}"
    return int(same.sum())


def paths_diverge(orc_hit, gpu_hit, rows=None):
    """True when some (flagged) path took a different hit on the two sides."""
    if rows is not None:
        gpu_hit = gpu_hit[rows]
    return not np.array_equal(orc_hit, gpu_hit)


def check_counts(orc_count, orc_flagged, gpu_count, gpu_flagged=None, diverged=True):
    allowance = np.concatenate([[0], np.cumsum(orc_flagged)[:-1]])
    diff = np.abs(np.asarray(gpu_count, np.int64) - np.asarray(orc_count, np.int64))
    assert (diff <= allowance).all(), f"counts {list(gpu_count)} vs {list(orc_count)}, allowance {list(allowance)}"
    if gpu_flagged is not None and not diverged:
        assert np.array_equal(np.asarray(gpu_flagged, np.int64), np.asarray(orc_flagged, np.int64)), \
            f"flagged per generation {list(gpu_flagged)} vs {list(orc_flagged)}"


def check_mics(orc_es, orc_ef, gpu_es, gpu_ef, diverged=False):
    eo = orc_es + orc_ef
    eg = gpu_es + gpu_ef
    emax = max(eo.max(), 1e-300) if eo.size else 1e-300
    strict_orc = orc_ef == 0
    extra = strict_orc & (gpu_ef != 0)
    n_extra = int(extra.sum())
    assert diverged or n_extra == 0, \
        f"{n_extra} microphones with GPU flag energy where the oracle has none (no path diverged)"
    strict = strict_orc & ~extra
    big = strict & (eo > 1e-12 * emax)
    tiny = strict & ~big
    with np.errstate(divide="ignore"):
        ddb = np.abs(10 * np.log10(eg[big]) - 10 * np.log10(eo[big]))
    assert (ddb <= DB_TOL).all(), f"{int((ddb > DB_TOL).sum())} strict mics beyond {DB_TOL} dB (max {ddb.max()})"
    assert (eg[tiny] < 2e-12 * emax).all(), "energy where the oracle has none"
    s_o, s_g = eo[strict].sum(), eg[strict].sum()
    if s_o > 0:
        assert abs(s_g - s_o) <= REL_SUM_TOL * s_o, f"strict energy sum {s_g} vs {s_o}"
    ns = ~strict
    lim = NONSTRICT_REL * eo[ns] + gpu_ef[ns] + orc_ef[ns] + 1e-300
    assert (np.abs(eg[ns] - eo[ns]) <= lim).all(), "non-strict microphone outside its bound"
    energised = eo > 0
    return {"strict": int(strict.sum()), "nonstrict": int(ns.sum()), "max_db": float(ddb.max()) if ddb.size else 0.0,
            "nonzero": int(energised.sum()), "energised": int(energised.sum()),
            "strict_energised": int((strict & energised).sum()), "gpu_flag_only": n_extra}


def strict_share(m):
    """Fraction of the oracle's energised microphones that are strict."""
    return m["strict_energised"] / max(m["energised"], 1)
