"""GPU: launch knobs and their autotuner.  Knobs split the work differently over the chip and
must never change a result: every setting gives the default's outputs bit for bit, alone
and in a batch."""
import numpy as np
import pytest
import torch

from paper_2104_06800_amd import autotune, synth

pytestmark = pytest.mark.gpu

KEYS = ("idepth", "rigid", "pose", "conf", "stats", "idepth_coarse", "rigid_coarse")


@pytest.fixture(scope="module")
def lib():
    from paper_2104_06800_amd.binding import Voldor
    v = Voldor(0)
    yield v
    v.close()


def alloc(lib, w):
    return lib.alloc(w["params"], w["flow"], w["pose_init"], w.get("prior_idepth"), w.get("prior_pose"))


def host(b):
    torch.cuda.synchronize()
    return {k: b[k].cpu().numpy().copy() for k in KEYS}


SETTINGS = [dict(local_chains=1), dict(local_chains=2, local_spec=1), dict(local_chains=4, local_spec=3),
            dict(local_spec=8, coarse_spec=1), dict(coarse_spec=4, coarse_lanes=4), dict(coarse_lanes=16),
            dict(local_chains=2, local_spec=5, coarse_spec=3, coarse_lanes=16), dict(local_order=2),
            dict(local_order=1, local_chains=2), dict(local_order=2, local_chains=4, local_spec=3)]


@pytest.mark.parametrize("case", ["street_320x240", "indoor_prior_160x120", "plain_64x48"])
def test_knobs_leave_results_bit_identical(lib, case):
    w = {"street_320x240": lambda: synth.make_window(2, 11, H=240, W=320),
         "indoor_prior_160x120": lambda: synth.make_window(3, 12, H=120, W=160, N=5),
         "plain_64x48": lambda: synth.make_window(1, 13)}[case]()
    p = dict(w["params"], iters=3)
    lib.set_knobs(p, None)
    b = alloc(lib, w)
    lib.run(p, b, iters=3)
    ref = host(b)
    for kn in SETTINGS:
        print(f"{case}: knobs {kn}", flush=True)
        lib.set_knobs(p, kn)
        assert lib.get_knobs(p) == dict(dict(local_chains=0, local_spec=0, coarse_spec=0, coarse_lanes=0,
                                             local_order=0), **kn)
        b = alloc(lib, w)
        lib.run(p, b, iters=3)
        got = host(b)
        for k in KEYS:
            assert np.array_equal(got[k], ref[k], equal_nan=True), (kn, k)
    lib.set_knobs(p, None)
    assert lib.get_knobs(p) == dict(local_chains=0, local_spec=0, coarse_spec=0, coarse_lanes=0, local_order=0)


def test_batch_with_per_window_knobs_equals_individual_runs(lib):
    ws = [synth.make_window(1, 30), synth.make_window(3, 31, H=53, W=70, N=4), synth.make_window(2, 32, H=64, W=96)]
    knobs = (dict(local_chains=2, local_spec=3), dict(local_chains=1, coarse_spec=2, local_order=2), {})
    for w, kn in zip(ws, knobs):
        lib.set_knobs(w["params"], kn or None)
    single = [(w["params"], alloc(lib, w)) for w in ws]
    for p, b in single:
        lib.run(p, b, iters=2)
    batch = [(w["params"], alloc(lib, w)) for w in ws]
    lib.batch_run(batch, 2)
    for (_, x), (_, y) in zip(batch, single):
        hx, hy = host(x), host(y)
        for k in KEYS:
            assert np.array_equal(hx[k], hy[k], equal_nan=True), k
    for w in ws:
        lib.set_knobs(w["params"], None)


def test_bad_knobs_rejected(lib):
    from paper_2104_06800_amd.binding import VoldorError
    p = synth.make_window(1, 0)["params"]
    for bad in (dict(local_spec=9), dict(coarse_lanes=6), dict(local_chains=-1), dict(coarse_spec=-2),
                dict(local_order=3), dict(local_order=-1)):
        with pytest.raises(VoldorError):
            lib.set_knobs(p, bad)


def test_autotuner_keeps_results_and_caches(lib, tmp_path):
    w = synth.make_window(2, 14, H=192, W=320)
    w["params"]["iters"] = 2
    space = dict(local_chains=(2, 8), local_spec=(1, 2), coarse_spec=(4, 8), coarse_lanes=(8, 16))
    res = autotune.tune(lib, w, reps=1, space=space)
    print("autotune:", res)
    assert res["tried"] == 8 and res["ms"] <= res["default_ms"]
    path = str(tmp_path / "knobs.json")
    table = {autotune.bucket(w["params"]): res}
    autotune.save(table, path)
    lib.set_knobs(w["params"], None)
    assert autotune.apply(lib, autotune.load(path), [w["params"]]) == (1 if res["knobs"] else 0)
    assert {k: v for k, v in lib.get_knobs(w["params"]).items() if v} == res["knobs"]
    lib.set_knobs(w["params"], None)
