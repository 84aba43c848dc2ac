"""Shared checks of the GPU parity tests (test helpers; no test functions here)."""
import numpy as np

from oracle import gem as ogem
from oracle import geometry as geo

# FP32 energies of <= 12 terms agree with the FP64 oracle to ~1e-5 of their size; an argmin
# may differ from the oracle's only between slots closer than that.
TIE_TOL = 2e-5
# candidate values are formed in FP32 on the GPU (a few ulp from the FP64 oracle's)
MEMBER_TOL = 1e-5
# a flow sample position this close to the edge of the sampling grid (or a depth this close
# to the camera plane) is inside in one precision and outside in the other
EDGE_EPS = 1e-3


def position_bound(p):
    """Largest energy change (bits) that FP32 rounding of the flow sample positions can
    cause: a coordinate below max(W, H) is held to half an ulp, which the bilinear sample of a
    flow field with gradients up to ~2 px/px carries into the residual as up to 2 ulp; the MIE
    cost of a frame changes by at most 2 / (alpha ln 2) bits per px of residual (its slope at
    r = alpha for the log-logistic shape 2, the steepest there), and N frames add up."""
    ulp = np.spacing(np.float32(max(p["W"], p["H"])))
    return p["N"] * 2.0 / (p["fisk_alpha"] * np.log(2.0)) * 2.0 * float(ulp)


def on_validity_edge(p, ob, u, v, rho):
    """True where some flow term of pixel (u, v) at inverse depth rho takes its validity
    decision within rounding: the sample position p_{t-1} (t >= 2) within EDGE_EPS px of the
    grid boundary, or Q_z within EDGE_EPS of 0 in some frame."""
    u, v, rho = np.atleast_1d(u), np.atleast_1d(v), np.atleast_1d(rho).astype(np.float64)
    intr = (p["fx"], p["fy"], p["cx"], p["cy"])
    xt = geo.rays(u, v, *intr)
    edge = np.zeros(u.shape, dtype=bool)
    for t in range(p["N"]):
        R, tt = geo.pose_rt(ob["pose"][t])
        Q = geo.scaled_point(R, tt, xt, rho)
        edge |= np.abs(Q[..., 2]) <= EDGE_EPS
        if t < p["N"] - 1:                       # p_t is the sample position of term t + 2
            px, py, _ = geo.project(Q, *intr)
            for c, hi in ((px, p["W"] - 1), (py, p["H"] - 1)):
                edge |= (np.abs(c) <= EDGE_EPS) | (np.abs(c - hi) <= EDGE_EPS)
    return edge


def frac_close_rel(a, b, rel=1e-3):
    return float(np.mean(np.abs(a - b) <= rel * np.abs(b)))


def check_mstep(p, ob, rho_before, gpu_rho, level, it, groups=None, frac_bar=None, report=None):
    """M-step check on the pixels of `groups` (default: every chain of the level).

    ob          oracle buffers holding the state the M-step used (q, poses, priors, coarse
                values); their level result is the oracle's own sweep
    rho_before  full-resolution inverse depth both sides started from
    gpu_rho     the GPU's result on the level grid

    Where energies are flat to FP32 resolution several slots are correct, and once one pixel
    of a chain takes another of them, the predecessor slot of the pixels after it differs
    too.  So every pixel is checked against its own candidate set, rebuilt with the oracle:
    slot 0 the current value, slot 1 the GPU's result at the chain predecessor (the current
    value at the chain head), slot 2 the coarse value (local level), slots 3..K-1 the Philox
    draws.  The GPU's value must be one of them, and its oracle energy must be within
    TIE_TOL (1 + |E|) of the set's minimum, unless one of the two competing values puts a
    flow term's validity decision on the edge of the sampling grid (within EDGE_EPS; FP32 and
    FP64 may decide it differently), or the excess is within position_bound (FP32 rounding of
    the sample positions on a noisy flow field); at most max(2, 0.1%) of the pixels may be
    such cases.
    Exact agreement with the oracle's own sweep is returned (and asserted when frac_bar is
    given).  With a dict as `report`, it also receives measured reasons for disagreement:
      flat        fraction of pixels whose candidate set under the oracle's own sweep (its
                  predecessor value in slot 1) has a second distinct value within TIE_TOL of
                  the best energy: both are correct picks there
      disagree    fraction of pixels differing from the oracle's sweep by more than 1e-3
      cascade     fraction of those disagreements whose chain predecessor already differed
                  (the predecessor slot is then another value on the two sides)
      flat_first  fraction of those disagreements whose predecessor agreed (so both sides
                  had the same candidates): each is a flat pixel by the validity check
    Returns (fraction agreeing with the oracle to 1e-3, pixels checked)."""
    lv = ogem.Level(p, level)
    coarse = level == ogem.COARSE
    key = "idepth_coarse" if coarse else "idepth"
    ref = np.asarray(ob[key], dtype=np.float64).ravel()
    got = np.asarray(gpu_rho, dtype=np.float64).ravel()
    if groups is None:
        groups = ogem.chains(p, level, it % 4)
    w = ogem.Window(p, ob)
    K = p["n_candidates"]
    q = np.asarray(ob["rigid_coarse" if coarse else "rigid"], dtype=np.float64).reshape(w.N, -1)
    rho_cur = np.asarray(rho_before, dtype=np.float64).ravel()[lv.full]
    if not coarse:
        s = p["coarse_stride"]
        hc, wc = ogem.lattice_shape(p["H"], p["W"], s)
        rc_all = np.asarray(ob["idepth_coarse"], dtype=np.float64)[np.minimum(lv.v // s, hc - 1),
                                                                   np.minimum(lv.u // s, wc - 1)]
    checked = 0
    edge_cases = 0
    pos_tol = position_bound(p)
    n_flat = n_dis = n_casc = 0
    for g in groups:
        n, L = g.shape
        flat = g.ravel()
        cur = rho_cur[g]
        pred = np.concatenate([cur[:, :1], got[g[:, :-1]]], axis=1)
        slot2 = cur if coarse else rc_all[g]
        rand = ogem.candidates_random(p, lv, it, level, rho_cur[flat], flat).reshape(n, L, -1)
        opred = np.concatenate([cur[:, :1], ref[g[:, :-1]]], axis=1)
        cand = np.concatenate([cur[..., None], pred[..., None], slot2[..., None], rand, got[g][..., None],
                               opred[..., None]], axis=2)
        qhat = w.prior_posteriors(lv.u[flat], lv.v[flat], rho_cur[flat])
        E = w.energy(lv.u[flat], lv.v[flat], cand.reshape(n * L, K + 2), q[:, flat], qhat).reshape(n, L, K + 2)
        # the oracle's own candidate set: its sweep's predecessor value in slot 1
        oset = np.concatenate([cand[..., :1], cand[..., K + 1:], cand[..., 2:K]], axis=2)
        oE = np.concatenate([E[..., :1], E[..., K + 1:], E[..., 2:K]], axis=2)
        if coarse:
            oE[..., 2] = np.inf
        ob_best = oE.min(axis=2)
        vbest = np.take_along_axis(oset, np.argmin(oE, axis=2)[..., None], axis=2)
        other = np.abs(oset - vbest) > MEMBER_TOL * np.abs(vbest)
        second = np.where(other, oE, np.inf).min(axis=2)
        is_flat = second - ob_best <= TIE_TOL * (1.0 + np.abs(ob_best))
        dis = np.abs(got[g] - ref[g]) > 1e-3 * np.abs(ref[g])
        pdiff = np.abs(pred - opred) > 1e-3 * np.abs(opred)
        n_flat += int(is_flat.sum())
        n_dis += int(dis.sum())
        n_casc += int((dis & pdiff).sum())
        E = E[..., :K + 1]
        if coarse:
            E[..., 2] = np.inf
        best = E[..., :K].min(axis=2)
        eg = E[..., K]
        over = eg - best - TIE_TOL * (1.0 + np.abs(best))
        near = np.abs(cand[..., :K] - got[g][..., None]) <= MEMBER_TOL * np.abs(cand[..., :K])
        if coarse:
            near[..., 2] = False
        member = near.any(axis=2)
        bad = (over > 0) | ~member
        for a, i in np.argwhere(bad):
            # a validity decision taken on the grid edge makes both choices correct, and so
            # does an excess that FP32 sample positions can produce
            j = g[a, i]
            kb = int(np.argmin(E[a, i, :K]))
            if member[a, i] and (over[a, i] <= pos_tol or on_validity_edge(
                    p, ob, lv.u[[j, j]], lv.v[[j, j]], np.array([got[j], cand[a, i, kb]])).any()):
                bad[a, i] = False
                edge_cases += 1
        if bad.any():
            a, i = np.argwhere(bad)[0]
            j = g[a, i]
            raise AssertionError(
                f"pixel {j} (node {i} of a chain): GPU value {got[j]:.7g} with E={eg[a, i]:.9g} "
                f"{'is not one of its candidates' if not member[a, i] else 'is not a tie'}; "
                f"best E={best[a, i]:.9g} at {cand[a, i, np.argmin(E[a, i, :K])]:.7g}; oracle's sweep {ref[j]:.7g}")
        checked += flat.size
    assert edge_cases <= max(2, 1e-3 * checked), f"{edge_cases} validity-edge or rounding cases in {checked} pixels"
    pix_all = np.concatenate([g.ravel() for g in groups])
    frac = frac_close_rel(got[pix_all], ref[pix_all])
    if report is not None:
        report.update(flat=n_flat / max(checked, 1), disagree=n_dis / max(checked, 1),
                      cascade=n_casc / max(n_dis, 1), flat_first=(n_dis - n_casc) / max(n_dis, 1),
                      pixels=checked)
    if frac_bar is not None:
        assert frac >= frac_bar, f"only {frac:.4f} of M-step results agree with the oracle's sweep"
    return frac, checked
