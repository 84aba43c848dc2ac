"""GPU parity of the learned-proposal kernels against the FP64 oracle (oracle/proposal.py).

Both sides see the same BF16 values (inputs, weights, upstream gradients); the kernels sum
their products in FP32.  Bars:
  one layer (forward, dx, dw, db)  |gpu - oracle| <= 1e-5 * (sum of |terms|) elementwise:
                                   an FP32 sum of K <= 1152 terms errs by ~sqrt(K) 2^-24 of it
  BF16 outputs                     exactly the round-to-nearest-even of the GPU's own FP32 value
  whole network (logits)           6 layers with BF16 activations between them: a rounding that
                                   lands on the other side of a midpoint moves one activation by
                                   one BF16 ulp (2^-8 relative), so the logits may differ by
                                   <= 1e-2 of their scale at a few pixels and <= 1e-4 on average
  training step                    loss rel 1e-4; per-layer gradients ||gpu - oracle|| <= 2e-2
                                   ||oracle|| (upstream gradients are stored in BF16 between
                                   layers: 2^-9 relative per element, five stages); Adam on the
                                   GPU's gradients rel 1e-5 of the step; BF16 copies exact
"""
import numpy as np
import pytest
import torch

from oracle import proposal as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2104_06800_amd.binding import Voldor
    v = Voldor(0)
    yield v
    v.close()


def bits(a):
    """BF16 bit patterns (int16 tensor on the GPU) of the values a (rounded to nearest even)."""
    f = P.bf16(a).astype(np.float32)
    return torch.from_numpy((f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)).cuda()


def from_bits(t):
    u = t.detach().cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def np_(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


CASES = [
    dict(H=9, W=13, Cin=16, Cout=32, stride=1, up=0, relu=0, skip=False),
    dict(H=9, W=13, Cin=64, Cout=64, stride=2, up=0, relu=1, skip=False),
    dict(H=7, W=10, Cin=128, Cout=64, stride=1, up=1, relu=1, skip=True),
    dict(H=33, W=40, Cin=64, Cout=128, stride=1, up=0, relu=1, skip=False),
    dict(H=16, W=20, Cin=128, Cout=128, stride=2, up=0, relu=0, skip=False),
    # stride-1 halo tiles with ragged edges in both directions (4- and 8-row tiles of 32 columns)
    dict(H=37, W=70, Cin=128, Cout=128, stride=1, up=0, relu=1, skip=False),
    dict(H=21, W=45, Cin=64, Cout=32, stride=1, up=0, relu=0, skip=True),
    dict(H=13, W=34, Cin=128, Cout=64, stride=1, up=1, relu=1, skip=False),
    # stride-2 halo tiles (4 rows of 32 outputs, 9 x 65 source pixels) with ragged edges; a
    # 32-channel output takes the staged kernel
    dict(H=37, W=131, Cin=64, Cout=128, stride=2, up=0, relu=1, skip=False),
    dict(H=22, W=70, Cin=16, Cout=64, stride=2, up=0, relu=0, skip=True),
    dict(H=21, W=45, Cin=16, Cout=32, stride=2, up=0, relu=1, skip=False),
]


def case_data(c, seed):
    rng = np.random.default_rng(seed)
    x = P.bf16(rng.normal(size=(c["H"], c["W"], c["Cin"])))
    w = P.bf16(rng.normal(scale=0.1, size=(c["Cout"], 3, 3, c["Cin"])))
    b = rng.normal(scale=0.1, size=c["Cout"]).astype(np.float32).astype(np.float64)
    return x, w, b, rng


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"{c['H']}x{c['W']}_{c['Cin']}to{c['Cout']}_s{c['stride']}_up{c['up']}")
def test_conv_forward(lib, c):
    x, w, b, rng = case_data(c, 1)
    ref = P.conv3x3(x, w, b, c["stride"], bool(c["up"]))
    scale = P.conv3x3(np.abs(x), np.abs(w), np.abs(b), c["stride"], bool(c["up"]))
    skip_t = None
    if c["skip"]:
        skip = P.bf16(rng.normal(size=ref.shape))
        ref, scale, skip_t = ref + skip, scale + np.abs(skip), bits(skip)
    if c["relu"]:
        ref = np.maximum(ref, 0.0)
    y, yf = lib.conv3x3_bf16(bits(x), bits(w), torch.tensor(b, dtype=torch.float32).cuda(), skip_t,
                             stride=c["stride"], up=c["up"], relu=c["relu"])
    got = np_(yf)
    assert got.shape == ref.shape
    err = np.abs(got - ref) / (scale + 1e-30)
    print(f"max error / sum|terms| = {err.max():.2e}")
    assert err.max() <= 1e-5
    np.testing.assert_array_equal(from_bits(y), P.bf16(got))


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"{c['H']}x{c['W']}_{c['Cin']}to{c['Cout']}_s{c['stride']}_up{c['up']}")
def test_conv_backward(lib, c):
    x, w, b, rng = case_data(c, 2)
    y = P.conv3x3(x, w, b, c["stride"], bool(c["up"]))
    dy = P.bf16(rng.normal(size=y.shape))
    dx, dw, db = P.conv3x3_backward(x, w, dy, c["stride"], bool(c["up"]))
    sx, sw, sb = P.conv3x3_backward(np.abs(x), np.abs(w), np.abs(dy), c["stride"], bool(c["up"]))
    w_t = np.ascontiguousarray(np.transpose(w, (3, 1, 2, 0)))
    gx, gw, gb = lib.conv3x3_bf16_backward(bits(x), bits(w_t), bits(dy), stride=c["stride"], up=c["up"])
    for name, g, r, s in (("dx", gx, dx, sx), ("dw", gw, dw, sw), ("db", gb, db, sb)):
        e = np.abs(np_(g) - r) / (s + 1e-30)
        print(f"{name}: max error / sum|terms| = {e.max():.2e}")
        assert e.max() <= 1e-5, name


def params_and_window(seed=3, N=6, H=32, W=48):
    rng = np.random.default_rng(seed)
    params = P.init_params(seed, N)
    for k in params:
        if k.endswith(".b"):
            params[k] = rng.normal(scale=0.05, size=params[k].shape)
    params = {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}
    flow = rng.normal(scale=6.0, size=(N, H, W, 2)).astype(np.float32)
    flow[0, 3, 5, 0] = np.nan
    return params, flow, rng


def flat(params):
    out = []
    for name, _, _, _, _, _, _ in P.LAYERS:
        out += [params[name + ".w"].ravel(), params[name + ".b"].ravel()]
    return np.concatenate(out)


def unflat(vec):
    out, o = {}, 0
    for name, ci, co, _, _, _, _ in P.LAYERS:
        n = co * 9 * ci
        out[name + ".w"] = vec[o:o + n].reshape(co, 3, 3, ci)
        out[name + ".b"] = vec[o + n:o + n + co]
        o += n + co
    return out


def test_network_forward(lib):
    params, flow, _ = params_and_window()
    N, H, W, _ = flow.shape
    net = lib.net_alloc(flat(params))
    rho, q, o = lib.proposal_forward(net, torch.from_numpy(flow).cuda(), 1.7, 0.005, 0.5, logits=True)
    acts = P.forward(params, P.features(flow.astype(np.float64)), round_bf16=True)
    ref = acts["o"]
    got = np_(o)
    scale = np.abs(ref).max()
    d = np.abs(got - ref)
    print(f"logits: max |d| {d.max() / scale:.2e} of scale, mean {d.mean() / scale:.2e}")
    assert d.max() <= 1e-2 * scale and d.mean() <= 1e-4 * scale
    rr, qr = P.heads(got.astype(np.float64), N, 1.7, 0.005, 0.5)
    np.testing.assert_allclose(np_(rho), rr, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(np_(q), qr, rtol=1e-5, atol=1e-6)
    # the heads are fused into the last layer: without the logits they are the same bits
    rho2, q2, _ = lib.proposal_forward(net, torch.from_numpy(flow).cuda(), 1.7, 0.005, 0.5)
    assert np.array_equal(np_(rho2), np_(rho)) and np.array_equal(np_(q2), np_(q))


def test_conv_rejects_unaligned_bf16_arrays(lib):
    """The single-layer entry points read BF16 arrays as 16-byte vectors: a view 2 bytes off
    an allocation is rejected with EINVAL before any launch, forward and backward."""
    from paper_2104_06800_amd.binding import VoldorError
    c = CASES[0]
    x, w, b, rng = case_data(c, 5)
    xb, wb = bits(x), bits(w)

    def shifted(t):
        big = torch.zeros(t.numel() + 8, dtype=torch.int16, device="cuda")
        v = big[1:1 + t.numel()].view(t.shape)
        v.copy_(t)
        return v

    with pytest.raises(VoldorError, match="16-byte aligned"):
        lib.conv3x3_bf16(shifted(xb), wb, None)
    with pytest.raises(VoldorError, match="16-byte aligned"):
        lib.conv3x3_bf16(xb, shifted(wb), None)
    dy = bits(P.bf16(rng.normal(size=(c["H"], c["W"], c["Cout"]))))
    w_t = bits(np.ascontiguousarray(np.transpose(w, (3, 1, 2, 0))))
    with pytest.raises(VoldorError, match="16-byte aligned"):
        lib.conv3x3_bf16_backward(xb, w_t, shifted(dy))
    y, yf = lib.conv3x3_bf16(xb, wb, None)          # the aligned call still works
    assert y is not None and torch.isfinite(yf).all()


def test_training_step(lib):
    params, flow, rng = params_and_window(seed=4, N=3, H=24, W=32)
    N, H, W, _ = flow.shape
    rho_t = rng.uniform(0.01, 0.4, size=(H, W)).astype(np.float32)
    q_t = rng.uniform(0, 1, size=(N, H, W)).astype(np.float32)
    mask = (rng.uniform(size=(H, W)) < 0.7)
    tn, lam, lr = 1.3, 0.5, 1e-3
    net = lib.net_alloc(flat(params), train=True)
    loss = torch.zeros(3, dtype=torch.float64, device="cuda")
    cu = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()
    lib.proposal_train_step(net, cu(flow), tn, cu(rho_t), cu(q_t), cu(mask.astype(np.uint8), torch.uint8), lam, lr,
                            1, loss)
    acts = P.forward(params, P.features(flow.astype(np.float64)), round_bf16=True)
    L, do = P.loss(acts["o"], rho_t.astype(np.float64), q_t.astype(np.float64), tn, mask, lam)
    got_loss = np_(loss)
    print("loss", got_loss, L)
    assert got_loss[0] == pytest.approx(L, rel=1e-4)
    rparams = {k: (P.bf16(v) if k.endswith(".w") else v) for k, v in params.items()}
    grads = P.backward(rparams, acts, do)
    g_gpu = unflat(np_(net["grads"]))
    for k in grads:
        rel = np.linalg.norm(g_gpu[k] - grads[k]) / max(np.linalg.norm(grads[k]), 1e-30)
        print(f"grad {k}: relative error {rel:.2e}")
        assert rel <= 2e-2, k
    # Adam on the GPU's own gradients
    p0 = {k: v.copy() for k, v in params.items()}
    m = {k: np.zeros_like(v) for k, v in p0.items()}
    v2 = {k: np.zeros_like(v) for k, v in p0.items()}
    P.adam_step(p0, g_gpu, m, v2, 1, lr)
    new = unflat(np_(net["params"]))
    for k in p0:
        assert np.abs(new[k] - p0[k]).max() <= 1e-5 * lr + 1e-7 * np.abs(p0[k]).max(), k
    # BF16 copies follow the new parameters
    newflat = np_(net["params"])
    np.testing.assert_array_equal(from_bits(net["wbf16"]), P.bf16(newflat))
    wt = unflat(from_bits(net["wt_bf16"]))
    for name, ci, co, _, _, _, _ in P.LAYERS:
        t = wt[name + ".w"].reshape(-1)[:co * 9 * ci].reshape(ci, 3, 3, co)
        np.testing.assert_array_equal(np.transpose(t, (3, 1, 2, 0)), P.bf16(new[name + ".w"]))


def test_network_rejects_odd_sizes(lib):
    from paper_2104_06800_amd.binding import VoldorError
    params, flow, _ = params_and_window(N=2, H=8, W=10)
    net = lib.net_alloc(flat(params))
    with pytest.raises(VoldorError):
        lib.proposal_forward(net, torch.from_numpy(flow[:, :7]).contiguous().cuda(), 1.0, 0.01, 1.0)


# ----------------------------------------------------------------------------- learned start
WEIGHTS = __import__("os").path.join(__import__("os").path.dirname(__import__("os").path.dirname(
    __import__("os").path.abspath(__file__))), "paper_2104_06800_amd", "weights", "proposal_n6.npz")


def _host(b, keys=("idepth", "rigid", "pose", "conf", "stats")):
    torch.cuda.synchronize()
    return {k: b[k].cpu().numpy().copy() for k in keys}


def test_nan_weights_fall_back_to_plain_gem(lib):
    """Unusable network output (NaN weights): the start falls back to the random start and
    the run continues to plain GEM's full schedule, equal to plain GEM bit for bit."""
    from paper_2104_06800_amd import proposal as pr, synth
    w = synth.make_window(4, 1_000_100, H=96, W=128)
    p = w["params"]
    params = np.full(pr.init_params(0, p["N"]).shape, np.nan, dtype=np.float32)
    net = lib.net_alloc(params)
    a = lib.alloc(p, w["flow"], w["pose_init"])
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert pr.learned_run(lib, net, p, a, 4, fallback=fb)
    assert int(fb.cpu()[0]) == 1
    b = lib.alloc(p, w["flow"], w["pose_init"])
    lib.run(p, b, iters=p["iters"])
    ha, hb = _host(a), _host(b)
    for k in ha:
        assert np.array_equal(ha[k], hb[k]), k


def test_trained_start_does_not_fall_back_and_batch_matches(lib):
    """The trained network's start on windows of several shapes (one odd-sized, which takes
    the random start) in one batched, graph-captured run equals the per-window calls bit for
    bit, with the fallback flags of the per-window calls."""
    from paper_2104_06800_amd import proposal as pr, synth
    params, _ = pr.load(WEIGHTS)
    net = lib.net_alloc(params)
    ws = [synth.make_window(4, 1_000_200, H=96, W=128), synth.make_window(2, 1_000_201, H=80, W=160, N=4),
          synth.make_window(3, 1_000_202, H=64, W=96, N=5), synth.make_window(1, 1_000_203, H=45, W=64)]
    iters = 3
    single, flags = [], []
    for w in ws:
        p = w["params"]
        b = lib.alloc(p, w["flow"], w["pose_init"], w.get("prior_idepth"), w.get("prior_pose"))
        fb = torch.zeros(1, dtype=torch.int32, device="cuda")
        if p["H"] % 2 == 0 and p["W"] % 2 == 0:
            lib.proposal_start(net, p, b, fb)
        else:
            lib.init_idepth(p, b)
            fb.fill_(1)
        lib.run(p, b, iters=iters, init=False)
        single.append(_host(b))
        flags.append(int(fb.cpu()[0]))
    assert flags == [0, 0, 0, 1]
    batch = [(w["params"], lib.alloc(w["params"], w["flow"], w["pose_init"], w.get("prior_idepth"),
                                     w.get("prior_pose"))) for w in ws]
    fbs = torch.full((len(ws),), -1, dtype=torch.int32, device="cuda")
    for rep in range(2):                          # capture, then replay
        lib.batch_run_learned(net, batch, iters, fallback=fbs)
        assert fbs.cpu().tolist() == flags
        for (_, b), ref in zip(batch, single):
            got = _host(b)
            for k in got:
                assert np.array_equal(got[k], ref[k]), k
        for (p, b), w in zip(batch, ws):
            b["pose"].copy_(torch.as_tensor(w["pose_init"], dtype=torch.float64))


def test_learned_start_reaches_plain_error_in_fewer_ms(lib):
    """What the trained network gains on held-out 640x480 street windows (seeds not used in
    training): GEM from the network's start reaches plain GEM's median static inverse-depth
    error (median over windows, after median scaling) with fewer iterations, and in fewer
    wall-clock ms including the network."""
    from paper_2104_06800_amd import proposal as pr
    params, _ = pr.load(WEIGHTS)
    net = lib.net_alloc(params)
    test = pr.generate(list(range(pr.TEST_SEED0, pr.TEST_SEED0 + 12)), 12)
    print(f"learned gain: {len(test)} held-out windows", flush=True)
    summ = pr.summarize(pr.compare(lib, net, test, warm=False))
    print("learned gain:", {k: v for k, v in summ.items() if k != "err_learned_by_iters"})
    print("error by iterations:", np.round(summ["err_learned_by_iters"], 4))
    assert summ["iters_to_plain"] is not None and summ["iters_to_plain"] < 10
    assert summ["ms_to_plain_error"] < summ["ms_plain"]
    assert summ["err_learned_full"] < summ["err_plain"]
