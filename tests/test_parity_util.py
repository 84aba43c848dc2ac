"""CPU checks of the M-step parity checker itself: it accepts the oracle's own result and
rejects a planted non-tie divergence."""
import numpy as np
import pytest

from oracle import gem as ogem
from paper_2104_06800_amd import synth
from parity_util import check_mstep


def run_mstep(level, it=1):
    w = synth.make_window(1, 7, H=24, W=32, N=2)
    p = w["params"]
    ob = ogem.alloc_buffers(p, w["flow"], w["pose_gt"])
    ogem.init_idepth(p, ob)
    if level == ogem.LOCAL:
        ogem.rigidness_fb(p, ob, it, ogem.COARSE)
        ogem.depth_update(p, ob, it, ogem.COARSE)
    ogem.rigidness_fb(p, ob, it, level)
    rb = ob["idepth"].copy()
    ogem.depth_update(p, ob, it, level)
    key = "idepth_coarse" if level == ogem.COARSE else "idepth"
    return p, ob, rb, ob[key].copy()


@pytest.mark.parametrize("level", [0, 1])
def test_checker_accepts_identical_result(level):
    p, ob, rb, res = run_mstep(level)
    rep = {}
    frac, n = check_mstep(p, ob, rb, res.astype(np.float32), level, 1, report=rep)
    assert frac == 1.0 and n == res.size
    assert rep["disagree"] == 0.0 and rep["cascade"] == 0.0 and 0.0 <= rep["flat"] < 0.5


def test_checker_rejects_a_planted_worse_choice():
    p, ob, rb, res = run_mstep(1)
    bad = res.copy().ravel()
    chain = ogem.chains(p, 1, 1)[0][3]          # some chain; plant at its first pixel
    j = chain[0]
    bad[j] = np.clip(bad[j] * 1.7, p["idepth_min"], p["idepth_max"])
    with pytest.raises(AssertionError, match="not one of its candidates|not a tie"):
        check_mstep(p, ob, rb, bad.reshape(res.shape), 1, 1)


def test_checker_rejects_a_worse_candidate_from_the_set():
    """A value from the pixel's own candidate set that is clearly not minimal."""
    p, ob, rb, res = run_mstep(1)
    lv = ogem.Level(p, 1)
    chain = ogem.chains(p, 1, 1)[0][5]
    j = chain[0]
    rand = ogem.candidates_random(p, lv, 1, 1, rb.ravel()[lv.full][[j]], np.array([j]))[0]
    w = ogem.Window(p, ob)
    qh = w.prior_posteriors(lv.u[[j]], lv.v[[j]], rb.ravel()[lv.full][[j]])
    E = w.energy(lv.u[[j]], lv.v[[j]], rand[None], ob["rigid"].reshape(p["N"], -1)[:, [j]], qh)[0]
    worst = rand[np.argmax(E)]
    bad = res.copy().ravel()
    bad[j] = worst
    with pytest.raises(AssertionError, match="not a tie"):
        check_mstep(p, ob, rb, bad.reshape(res.shape), 1, 1)
