"""Bars for FP32 iterations against the FP64 oracle (shared by the GPU
parity tests).

The FP32 iteration (gm_opts.estep_fp64 = 0) is the FP64 iteration perturbed
by roundings at every operation.  FP64 iterations take every decision of the
oracle exactly and agree to rounding (test_gpu_fp64_exact); what FP32
rounding can legitimately move decides the bars here:

* Decisions.  K is compared exactly, except in cells flagged on either
  side NEAR_TIE (an annihilation decision within 1e-5 T/2 of the threshold
  of eq. omegak) or COV_FLOOR (a covariance that stopped factoring during
  the sweeps and got the eps I floor): whether a nearly singular covariance
  still factors is decided at the rounding level, and the floored fit then
  takes its own path.
* Parameters and likelihood.  The FP32 result is held to 1e-4 (parameters:
  |d omega|, |d mu| / sqrt(tr C / D), |d Sigma|_F / |Sigma|_F; L_pen and
  L_final: relative to max(|L|, N)), or to the resolution the cell itself
  gives them where that is coarser, taken from the oracle alone as the
  larger of
    - twice the oracle's own movement over the 50 sweeps after the compared
      sweep (the 50 before it when K changes within the 50 after): a cell
      stopped by the sweep cap, or by a stop test that fires on a slow drift,
      is not at a fixed point, and FP32 rounding shifts where along that
      drift it stands;
    - ten times the movement the oracle's FP32-rounding perturbation gives
      (oracle.MODE_ROUND32: each update's responsibilities and the updated
      component rounded to binary32): how far rounding at FP32 resolution
      moves this fit when iterated (flat directions of the penalised
      likelihood amplify it); the GPU rounds at more places than the model
      (exponentials, reciprocals, FP32 sums), hence the factor.
  Cells where K changes within both 50-sweep windows are compared on K and
  L only, and counted.
* Likelihood normalisation.  eq. (lnL-GM) with weights normalised to sum N
  depends on the velocity unit: scaling v by s subtracts N D ln s
  (test_likelihood_shifts_with_the_velocity_unit), so |L| has no unit-free
  size and can sit near zero; errors are taken relative to max(|L|, N):
  relative to |L| where the likelihood is large, and to one nat per
  particle (a unit change of ln s = 1/D) where it is small.
* Moments and the conservation of every output mixture are FP64 on both
  sides: 1e-12.
"""
import numpy as np

import oracle

from gpu_util import conservation, mixture_errors

NEAR = oracle.STATUS["NEAR_TIE"]
FLOOR = oracle.STATUS["COV_FLOOR"]
MOVE_SWEEPS = 50
ROUND32_FACTOR = 10.0


def _errs(a, b, c, D):
    if a["K"][c] != b["K"][c] or b["K"][c] == 0:
        return np.inf
    return max(mixture_errors(a, b, c, D))


def _lerr(a, b, c, n):
    vals = (a["L_pen"][c], b["L_pen"][c], a["L_final"][c], b["L_final"][c])
    if not all(np.isfinite(vals)):
        return 0.0 if vals[0] == vals[1] and vals[2] == vals[3] else np.inf
    return max(abs(vals[0] - vals[1]), abs(vals[2] - vals[3])) / max(abs(vals[1]), n)


def resolution(d, kmax, seed, sweeps, ref, **kw):
    """Per-cell resolution of the oracle's record `ref` at `sweeps`: returns
    (parameter bar, L bar) arrays before the 1e-4 floor; inf where K changes
    within both 50-sweep windows."""
    D = 1 if d["v"].ndim == 1 else d["v"].shape[1]
    n = np.diff(d["cell_off"]).astype(np.float64)
    n_cells = len(ref["K"])
    mode = kw.pop("mode", 0)
    nxt = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=kmax, seed=seed, max_sweeps=10000,
                          fixed_sweeps=sweeps + MOVE_SWEEPS, mode=mode, **kw)
    move = np.array([_errs(nxt, ref, c, D) for c in range(n_cells)])
    lmove = np.array([_lerr(nxt, ref, c, n[c]) if np.isfinite(move[c]) else np.inf for c in range(n_cells)])
    back = np.isinf(move) & (sweeps > MOVE_SWEEPS)
    if back.any():
        prv = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=kmax, seed=seed, max_sweeps=10000,
                              fixed_sweeps=np.where(back, sweeps - MOVE_SWEEPS, 1), mode=mode, **kw)
        for c in np.nonzero(back)[0]:
            move[c] = _errs(prv, ref, c, D)
            lmove[c] = _lerr(prv, ref, c, n[c]) if np.isfinite(move[c]) else np.inf
    r32 = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=kmax, seed=seed, max_sweeps=10000,
                          fixed_sweeps=sweeps, mode=mode | oracle.MODE_ROUND32, **kw)
    p32 = np.array([_errs(r32, ref, c, D) for c in range(n_cells)])
    l32 = np.array([_lerr(r32, ref, c, n[c]) for c in range(n_cells)])
    p32 = np.where(np.isfinite(p32), p32, 0.0)
    l32 = np.where(np.isfinite(l32), l32, 0.0)
    pbar = np.where(np.isfinite(move), np.maximum(2.0 * move, ROUND32_FACTOR * p32), np.inf)
    lbar = np.where(np.isfinite(lmove), np.maximum(2.0 * lmove, ROUND32_FACTOR * l32), np.inf)
    return pbar, lbar


def check(g, o, d, res, label, par_tol=1e-4, L_tol=1e-4, cells=None):
    """K exact outside NEAR_TIE and COV_FLOOR cells; moments and
    conservation 1e-12; parameters and L within max(tolerance, the cell's
    resolution) (res = resolution(...)).  Returns the parameter errors of
    the compared cells."""
    pres, lres = res
    D = 1 if d["v"].ndim == 1 else d["v"].shape[1]
    n = np.diff(d["cell_off"]).astype(np.float64)
    sel = range(len(o["K"])) if cells is None else list(cells)
    n_cells = len(sel)
    exempt = ((g["status"] | o["status"]) & (NEAR | FLOOR)).astype(bool)
    mism = [c for c in sel if g["K"][c] != o["K"][c] and not exempt[c]]
    assert not mism, (label, "K differs", mism, g["K"][mism], o["K"][mism])
    errs, lerrs, unsettled, wide, kdiff = [], [], 0, 0, 0
    for c in sel:
        scale = np.abs(o["moments"][c]).max()
        assert np.abs(g["moments"][c] - o["moments"][c]).max() <= 1e-12 * max(scale, 1e-300), (label, c)
        if g["K"][c] != o["K"][c]:
            kdiff += 1
            continue
        if o["K"][c] == 0:
            continue
        dw, dp, ds = conservation(g, c, D)
        assert max(dw, dp, ds) < 1e-12, (label, c, dw, dp, ds)
        if not (np.isfinite(o["L_pen"][c]) and np.isfinite(o["L_final"][c])):
            assert g["L_pen"][c] == o["L_pen"][c] and g["L_final"][c] == o["L_final"][c], (label, c)
            continue
        eL = _lerr(g, o, c, n[c])
        lerrs.append(eL)
        assert eL <= max(L_tol, lres[c]), (label, c, "L", g["L_pen"][c], o["L_pen"][c], g["L_final"][c],
                                           o["L_final"][c], "resolution", lres[c])
        if np.isinf(pres[c]):
            unsettled += 1
            continue
        e = max(mixture_errors(g, o, c, D))
        assert e <= max(par_tol, pres[c]), (label, c, "parameters", e, "resolution", pres[c])
        errs.append(e)
        wide += e > par_tol
    errs = np.array(errs if errs else [0.0])
    lerrs = np.array(lerrs if lerrs else [0.0])
    print("%s: %d cells, %d exempt (NEAR_TIE/COV_FLOOR), %d of them with another K; parameters compared in %d "
          "(%d unsettled): median %.1e p90 %.1e max %.1e, %d above %.0e and within the cell's resolution; "
          "L error median %.1e max %.1e of max(|L|, N), %d above %.0e" % (
              label, n_cells, exempt[sel].sum(), kdiff, len(errs), unsettled, np.median(errs),
              np.quantile(errs, 0.9), errs.max(), wide, par_tol, np.median(lerrs), lerrs.max(),
              (lerrs > L_tol).sum(), L_tol))
    return errs


STOP_RESOLUTION = 1e-5


def converged(g, d, kmax, seed, label, init=None, cells=None, **kw):
    """FP32 run to convergence against the oracle replayed to the GPU's own
    sweep counts.  The stop test compares relative changes of L of 1e-7,
    the size of FP32 rounding of L itself, so the stopping sweep can differ
    from the oracle's; the oracle's own change of L at the GPU's stopping
    sweep must then lie within STOP_RESOLUTION of max(|L|, N) (a hundred
    times the tolerance), and the records are compared with `check`.  A cell
    the GPU refitted from the cold start after rejecting its warm start is
    replayed from the cold start.  `cells` (optional) restricts the
    comparison to the non-empty cells of a sampled batch.  Returns the
    oracle's replay record."""
    n = np.diff(d["cell_off"])
    fs = np.maximum(g["sweeps"], 1)
    ini = None
    if init is not None:
        ini = {k: np.array(init[k]) for k in ("K", "omega", "mu", "sigma")}
        ini["K"][(g["status"] & oracle.STATUS["WARM_FALLBACK"]) != 0] = 0
    ot = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=kmax, seed=seed, max_sweeps=10000,
                         fixed_sweeps=fs, init=ini, **kw)
    prev = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=kmax, seed=seed, max_sweeps=10000,
                           fixed_sweeps=np.maximum(fs - 1, 1), init=ini, **kw)
    capped = (g["status"] & oracle.STATUS["MAXSWEEPS"]) != 0
    sel = np.arange(len(n)) if cells is None else np.asarray(cells)
    gaps = []
    for c in sel:
        if capped[c] or g["sweeps"][c] < 2 or g["K"][c] == 0 or ot["K"][c] != prev["K"][c]:
            continue
        gaps.append(abs(ot["L_pen"][c] - prev["L_pen"][c]) / max(abs(ot["L_pen"][c]), n[c]))
    gaps = np.array(gaps)
    print("%s: oracle's change of L at the GPU's stopping sweeps: median %.1e max %.1e of max(|L|, N)"
          % (label, np.median(gaps), gaps.max()))
    assert gaps.max() < STOP_RESOLUTION, (label, gaps.max())
    res = resolution(d, kmax, seed, fs, ot, init=ini, **kw)
    check(g, ot, d, res, label, cells=cells)
    return ot
