"""ctypes binding of libvoldor.so: the same entry points, argument marshalling only.

Every step of the method runs in the library's HIP kernels; PyTorch supplies device
memory (tensors) and the current HIP stream.  Importing this module loads the in-tree
library and fails loudly when it has not been built.
"""
import ctypes
import os

import torch

from .build import LIB

OK, EINVAL, ENOMEM, EDEVICE, ESINGULAR = 0, 1, 2, 3, 4
COARSE, LOCAL = 0, 1
RUN_INIT, RUN_NO_GRAPH = 1, 2
TIMER_LOCAL, TIMER_COARSE, TIMER_POSE = 0, 1, 2
NET_PARAMS = 470560
NOALLOC_SCRATCH_BYTES = 64 << 20
VC_OUT_LEN, VC_MAX_POSES = 5, 1024
SCORE_LEN = 29
STATS_LEN = 8
MAX_FRAMES, MAX_PRIORS = 8, 4


class VoldorError(RuntimeError):
    pass


class Window(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("N", ctypes.c_int32), ("P", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("fisk_alpha", ctypes.c_float), ("fisk_beta", ctypes.c_float),
                ("outlier_density", ctypes.c_float), ("hmm_gamma", ctypes.c_float),
                ("idepth_min", ctypes.c_float), ("idepth_max", ctypes.c_float), ("perturb_sigma0", ctypes.c_float),
                ("prior_sigma_rel", ctypes.c_float), ("prior_uniform_rel", ctypes.c_float),
                ("prior_inlier_default", ctypes.c_float),
                ("n_candidates", ctypes.c_int32), ("coarse_stride", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("pose_gn_steps", ctypes.c_int32), ("chain_axis", ctypes.c_int32), ("prior_model", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("window_id", ctypes.c_uint32), ("prior_disp_scale", ctypes.c_float),
                ("prior_fisk_beta", ctypes.c_float), ("init_random", ctypes.c_uint32)]


class Buffers(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("flow", "pose", "idepth", "rigid", "idepth_coarse", "rigid_coarse",
                 "prior_idepth", "prior_pose", "prior_weight", "conf", "stats")]


class Net(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("params", "wbf16", "wt_bf16", "adam_m", "adam_v", "grads")]


class AlignParams(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("robust", ctypes.c_int32), ("robust_scale", ctypes.c_float), ("gn_steps", ctypes.c_int32),
                ("normal_disc_rel", ctypes.c_float), ("scale_s", ctypes.c_float)]


EXPORTS = sorted(["voldor_ctx_create", "voldor_ctx_destroy", "voldor_last_error", "voldor_lattice_shape",
                  "voldor_init_idepth", "voldor_rigidness_fb", "voldor_depth_update", "voldor_level_step",
                  "voldor_pose_score", "voldor_pose_step", "voldor_gem_step", "voldor_finalize",
                  "voldor_run", "voldor_run_noalloc", "voldor_batch_run", "voldor_batch_run_learned",
                  "voldor_proposal_start", "voldor_timing", "voldor_timing_read",
                  "voldor_net_refresh", "voldor_proposal_forward", "voldor_proposal_train_step",
                  "voldor_conv3x3_bf16", "voldor_conv3x3_bf16_backward",
                  "voldor_align_p2p", "voldor_vc_scores", "voldor_set_knobs", "voldor_get_knobs",
                  "voldor_pose_sample", "voldor_align_sim3"])


class Knobs(ctypes.Structure):
    _fields_ = [("local_chains", ctypes.c_int32), ("local_spec", ctypes.c_int32),
                ("coarse_spec", ctypes.c_int32), ("coarse_lanes", ctypes.c_int32),
                ("local_order", ctypes.c_int32)]


class SampleParams(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int32), ("tries", ctypes.c_int32), ("sigma_w", ctypes.c_double),
                ("sigma_t_rel", ctypes.c_double), ("eps", ctypes.c_double)]


class VcParams(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("cell", ctypes.c_int32), ("conf_min", ctypes.c_float)]


def load_library(path=None):
    """Loads the C-ABI library: the in-tree build, or another build of the same sources
    (same ABI) named by the environment variable VOLDOR_LIBRARY."""
    path = path or os.environ.get("VOLDOR_LIBRARY") or LIB
    if not os.path.exists(path):
        raise VoldorError(f"{path} is missing: build it first (python -m paper_2104_06800_amd.build)")
    lib = ctypes.CDLL(path)
    P, I, V = ctypes.POINTER, ctypes.c_int, ctypes.c_void_p
    W, B = P(Window), P(Buffers)
    lib.voldor_ctx_create.argtypes = [P(V), I]
    lib.voldor_ctx_destroy.argtypes = [V]
    lib.voldor_ctx_destroy.restype = None
    lib.voldor_last_error.argtypes = [V]
    lib.voldor_last_error.restype = ctypes.c_char_p
    lib.voldor_lattice_shape.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         P(ctypes.c_int32), P(ctypes.c_int32)]
    lib.voldor_init_idepth.argtypes = [V, W, B, V]
    lib.voldor_rigidness_fb.argtypes = [V, W, B, I, I, V]
    lib.voldor_depth_update.argtypes = [V, W, B, I, I, V]
    lib.voldor_level_step.argtypes = [V, W, B, I, I, V]
    lib.voldor_pose_score.argtypes = [V, W, B, I, I, V, V, V]
    lib.voldor_pose_step.argtypes = [V, W, B, V]
    lib.voldor_gem_step.argtypes = [V, W, B, I, V]
    lib.voldor_finalize.argtypes = [V, W, B, I, V]
    lib.voldor_run.argtypes = [V, W, B, I, I, I, V]
    lib.voldor_run_noalloc.argtypes = [V, W, B, I, I, I, V]
    lib.voldor_batch_run.argtypes = [V, I, W, B, I, I, V]
    lib.voldor_batch_run_learned.argtypes = [V, P(Net), I, W, B, I, I, V, V]
    lib.voldor_proposal_start.argtypes = [V, P(Net), W, B, V, V]
    lib.voldor_timing.argtypes = [V, I]
    lib.voldor_set_knobs.argtypes = [V, W, P(Knobs)]
    lib.voldor_pose_sample.argtypes = [V, W, B, I, P(SampleParams), V, V, V]
    lib.voldor_get_knobs.argtypes = [V, W, P(Knobs)]
    lib.voldor_timing_read.argtypes = [V, I, P(ctypes.c_double), P(ctypes.c_int64)]
    F = ctypes.c_float
    lib.voldor_net_refresh.argtypes = [V, P(Net), V]
    lib.voldor_proposal_forward.argtypes = [V, P(Net), I, I, I, V, F, F, F, V, V, V, V]
    lib.voldor_proposal_train_step.argtypes = [V, P(Net), I, I, I, V, F, V, V, V, F, F, I, V, V]
    lib.voldor_conv3x3_bf16.argtypes = [V, I, I, I, I, I, I, I, V, V, V, V, V, V, V]
    lib.voldor_conv3x3_bf16_backward.argtypes = [V, I, I, I, I, I, I, V, V, V, V, V, V, V]
    lib.voldor_align_p2p.argtypes = [V, P(AlignParams), I, V, V, V, V, V, V, V, V]
    lib.voldor_align_sim3.argtypes = [V, P(AlignParams), I, V, V, V, V, V, V, V, V, V]
    lib.voldor_vc_scores.argtypes = [V, P(VcParams), V, V, I, V, ctypes.c_double, V, V, V]
    for n in EXPORTS:
        if n not in ("voldor_ctx_destroy", "voldor_last_error"):
            getattr(lib, n).restype = ctypes.c_int
    return lib


_LIB = load_library()


def lattice_shape(H, W, stride):
    hc, wc = ctypes.c_int32(), ctypes.c_int32()
    rc = _LIB.voldor_lattice_shape(H, W, stride, ctypes.byref(hc), ctypes.byref(wc))
    if rc:
        raise VoldorError(f"bad lattice {H}x{W} stride {stride}")
    return hc.value, wc.value


# window fields a parameter dict may leave out (the Gaussian-uniform prior model)
OPTIONAL_WINDOW_FIELDS = dict(prior_model=0, prior_disp_scale=0.0, prior_fisk_beta=1.0, init_random=0)


def make_window(p):
    """Window struct from a parameter dict (keys as in the struct)."""
    w = Window()
    for name, _ in Window._fields_:
        if name.startswith("reserved"):
            continue
        if name in OPTIONAL_WINDOW_FIELDS and name not in p:
            setattr(w, name, OPTIONAL_WINDOW_FIELDS[name])
            continue
        setattr(w, name, p[name] if name != "seed" else int(p[name]) & 0xFFFFFFFFFFFFFFFF)
    return w


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Voldor:
    """One library context on a device; methods mirror the C entry points."""

    def __init__(self, device=0):
        self.device = device
        h = ctypes.c_void_p()
        rc = _LIB.voldor_ctx_create(ctypes.byref(h), device)
        if rc:
            raise VoldorError(f"voldor_ctx_create: {_LIB.voldor_last_error(None).decode()}")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _LIB.voldor_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc:
            raise VoldorError(f"{what} -> {rc}: {_LIB.voldor_last_error(self._h).decode()}")

    # -- buffers ---------------------------------------------------------------
    def alloc(self, p, flow, pose, prior_idepth=None, prior_pose=None, prior_weight=None):
        """Device buffer set for one window; inputs are copied to the device."""
        dev = torch.device("cuda", self.device)
        H, W, N, P = p["H"], p["W"], p["N"], p.get("P", 0)
        hc, wc = lattice_shape(H, W, p["coarse_stride"])
        f32 = dict(dtype=torch.float32, device=dev)
        b = dict(
            flow=torch.as_tensor(flow, dtype=torch.float32).to(dev).contiguous(),
            pose=torch.as_tensor(pose, dtype=torch.float64).to(dev).contiguous(),
            idepth=torch.zeros((H, W), **f32), rigid=torch.zeros((N, H, W), **f32),
            idepth_coarse=torch.zeros((hc, wc), **f32), rigid_coarse=torch.zeros((N, hc, wc), **f32),
            prior_idepth=None, prior_pose=None, prior_weight=None,
            conf=torch.zeros((H, W), **f32), stats=torch.zeros(8, dtype=torch.float64, device=dev))
        if P:
            b["prior_idepth"] = torch.as_tensor(prior_idepth, dtype=torch.float32).to(dev).contiguous()
            b["prior_pose"] = torch.as_tensor(prior_pose, dtype=torch.float64).to(dev).contiguous()
            if prior_weight is not None:
                b["prior_weight"] = torch.as_tensor(prior_weight, dtype=torch.float32).to(dev).contiguous()
        return b

    def _bufs(self, p, b):
        H, W, N, P = p["H"], p["W"], p["N"], p.get("P", 0)
        hc, wc = lattice_shape(H, W, p["coarse_stride"])
        shapes = dict(flow=(N, H, W, 2), pose=(N, 6), idepth=(H, W), rigid=(N, H, W),
                      idepth_coarse=(hc, wc), rigid_coarse=(N, hc, wc), conf=(H, W), stats=(8,))
        if P:
            shapes.update(prior_idepth=(P, H, W), prior_pose=(P, 6))
            if b.get("prior_weight") is not None:
                shapes["prior_weight"] = (P, H, W)
        for k, shp in shapes.items():
            t = b.get(k)
            if t is None:
                raise VoldorError(f"buffer {k} missing")
            want = torch.float64 if k in ("pose", "prior_pose", "stats") else torch.float32
            if tuple(t.shape) != shp or t.dtype != want or not t.is_cuda or not t.is_contiguous():
                raise VoldorError(f"buffer {k}: need contiguous {want} {shp} on the GPU, got "
                                  f"{t.dtype} {tuple(t.shape)} cuda={t.is_cuda}")
        return Buffers(*[_ptr(b.get(n)) for n, _ in Buffers._fields_])

    # -- entry points -----------------------------------------------------------
    def init_idepth(self, p, b, stream=None):
        self._check(_LIB.voldor_init_idepth(self._h, make_window(p), self._bufs(p, b), _stream(stream)),
                    "voldor_init_idepth")

    def rigidness_fb(self, p, b, it, level, stream=None):
        self._check(_LIB.voldor_rigidness_fb(self._h, make_window(p), self._bufs(p, b), it, level,
                                             _stream(stream)), "voldor_rigidness_fb")

    def depth_update(self, p, b, it, level, stream=None):
        self._check(_LIB.voldor_depth_update(self._h, make_window(p), self._bufs(p, b), it, level,
                                             _stream(stream)), "voldor_depth_update")

    def level_step(self, p, b, it, level, stream=None):
        self._check(_LIB.voldor_level_step(self._h, make_window(p), self._bufs(p, b), it, level,
                                           _stream(stream)), "voldor_level_step")

    def pose_score(self, p, b, t, cand, stream=None):
        cand = torch.as_tensor(cand, dtype=torch.float64).to(b["pose"].device).reshape(-1, 6).contiguous()
        out = torch.zeros((cand.shape[0], SCORE_LEN), dtype=torch.float64, device=cand.device)
        self._check(_LIB.voldor_pose_score(self._h, make_window(p), self._bufs(p, b), t, cand.shape[0],
                                           _ptr(cand), _ptr(out), _stream(stream)), "voldor_pose_score")
        return out

    def pose_step(self, p, b, stream=None):
        self._check(_LIB.voldor_pose_step(self._h, make_window(p), self._bufs(p, b), _stream(stream)),
                    "voldor_pose_step")

    def gem_step(self, p, b, it, stream=None):
        self._check(_LIB.voldor_gem_step(self._h, make_window(p), self._bufs(p, b), it, _stream(stream)),
                    "voldor_gem_step")

    def finalize(self, p, b, it, stream=None):
        self._check(_LIB.voldor_finalize(self._h, make_window(p), self._bufs(p, b), it, _stream(stream)),
                    "voldor_finalize")

    def run(self, p, b, iters=None, init=True, first_iter=0, stream=None):
        """GEM window in one call: optional random init, iterations first_iter ..
        first_iter + iters - 1, finalize."""
        iters = p.get("iters", 5) if iters is None else iters
        self._check(_LIB.voldor_run(self._h, make_window(p), self._bufs(p, b), first_iter, iters,
                                    RUN_INIT if init else 0, _stream(stream)), "voldor_run")

    def run_noalloc(self, p, b, iters=None, init=True, first_iter=0, stream=None):
        """As run, with the library's static per-device scratch (no allocation)."""
        iters = p.get("iters", 5) if iters is None else iters
        self._check(_LIB.voldor_run_noalloc(self._h, make_window(p), self._bufs(p, b), first_iter, iters,
                                            RUN_INIT if init else 0, _stream(stream)), "voldor_run_noalloc")

    def batch_run(self, windows, iters, init=True, graph=True, stream=None):
        """windows: list of (params, buffers); every window runs iters iterations, batched
        launches captured in a HIP graph (replayed by identical later calls)."""
        n = len(windows)
        wins = (Window * n)(*[make_window(p) for p, _ in windows])
        bufs = (Buffers * n)(*[self._bufs(p, b) for p, b in windows])
        flags = (RUN_INIT if init else 0) | (0 if graph else RUN_NO_GRAPH)
        self._check(_LIB.voldor_batch_run(self._h, n, wins, bufs, iters, flags, _stream(stream)), "voldor_batch_run")

    def pose_sample(self, p, b, it, sp, stream=None):
        """The sampled pose M-step over frames 1..N (updates b["pose"]); sp: dict of
        SampleParams fields.  Returns (cov [N][36], info [N][4]) FP64 device tensors."""
        dev = b["pose"].device
        cov = torch.zeros((p["N"], 36), dtype=torch.float64, device=dev)
        info = torch.zeros((p["N"], 4), dtype=torch.float64, device=dev)
        s = SampleParams(**{k: sp[k] for k, _ in SampleParams._fields_})
        self._check(_LIB.voldor_pose_sample(self._h, make_window(p), self._bufs(p, b), it, ctypes.byref(s), _ptr(cov),
                                            _ptr(info), _stream(stream)), "voldor_pose_sample")
        return cov, info

    def set_knobs(self, p, knobs=None):
        """Launch knobs (dict of Knobs fields; None removes) for windows shaped like p."""
        k = None if knobs is None else ctypes.byref(Knobs(**{n: int(knobs.get(n, 0)) for n, _ in Knobs._fields_}))
        self._check(_LIB.voldor_set_knobs(self._h, make_window(p), k), "voldor_set_knobs")

    def get_knobs(self, p):
        k = Knobs()
        self._check(_LIB.voldor_get_knobs(self._h, make_window(p), ctypes.byref(k)), "voldor_get_knobs")
        return {n: getattr(k, n) for n, _ in Knobs._fields_}

    def batch_run_learned(self, net, windows, iters, graph=True, fallback=None, stream=None):
        """batch_run with every window started by the proposal network; fallback (int32
        device tensor [n] or None) receives 1 where a window took the random start."""
        n = len(windows)
        wins = (Window * n)(*[make_window(p) for p, _ in windows])
        bufs = (Buffers * n)(*[self._bufs(p, b) for p, b in windows])
        flags = 0 if graph else RUN_NO_GRAPH
        self._check(_LIB.voldor_batch_run_learned(self._h, ctypes.byref(self._net(net)), n, wins, bufs, iters, flags,
                                                  _ptr(fallback), _stream(stream)), "voldor_batch_run_learned")

    def proposal_start(self, net, p, b, fallback=None, stream=None):
        """The proposal network's start of window (p, b): writes b's idepth and rigid; fallback
        (int32 device tensor [1] or None) receives 1 where the random start replaced it."""
        self._check(_LIB.voldor_proposal_start(self._h, ctypes.byref(self._net(net)), make_window(p), self._bufs(p, b),
                                               _ptr(fallback), _stream(stream)), "voldor_proposal_start")

    def timing(self, enable, timers=(TIMER_LOCAL, TIMER_COARSE, TIMER_POSE)):
        """Starts (afresh) or stops the launch timers of the given classes."""
        mask = sum(1 << t for t in set(timers)) if enable else 0
        self._check(_LIB.voldor_timing(self._h, mask), "voldor_timing")

    def timing_read(self, timer):
        """(total ms, launches) of one timer class since the last read; waits for them."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(_LIB.voldor_timing_read(self._h, timer, ctypes.byref(ms), ctypes.byref(n)), "voldor_timing_read")
        return ms.value, n.value

    # -- learned proposal -------------------------------------------------------
    def net_alloc(self, params, train=False):
        """Device buffers of the proposal network from FP32 parameters [NET_PARAMS]."""
        dev = torch.device("cuda", self.device)
        p = torch.as_tensor(params, dtype=torch.float32).to(dev).contiguous()
        if p.numel() != NET_PARAMS:
            raise VoldorError(f"need {NET_PARAMS} parameters, got {p.numel()}")
        z16 = lambda: torch.zeros(NET_PARAMS, dtype=torch.int16, device=dev)
        net = dict(params=p, wbf16=z16(), wt_bf16=z16() if train else None,
                   adam_m=torch.zeros_like(p) if train else None, adam_v=torch.zeros_like(p) if train else None,
                   grads=torch.zeros_like(p) if train else None)
        self.net_refresh(net)
        return net

    @staticmethod
    def _net(net):
        return Net(*[_ptr(net.get(n)) for n, _ in Net._fields_])

    def net_refresh(self, net, stream=None):
        self._check(_LIB.voldor_net_refresh(self._h, ctypes.byref(self._net(net)), _stream(stream)),
                    "voldor_net_refresh")

    def proposal_forward(self, net, flow, tnorm, idepth_min, idepth_max, logits=False, stream=None):
        """flow [N][H][W][2] FP32 device tensor -> (idepth [H][W], rigid [N][H][W], logits or None)."""
        N, H, W, _ = flow.shape
        dev = flow.device
        rho = torch.empty((H, W), dtype=torch.float32, device=dev)
        q = torch.empty((N, H, W), dtype=torch.float32, device=dev)
        o = torch.empty((H, W, 32), dtype=torch.float32, device=dev) if logits else None
        self._check(_LIB.voldor_proposal_forward(self._h, ctypes.byref(self._net(net)), H, W, N, _ptr(flow),
                                                 float(tnorm), float(idepth_min), float(idepth_max), _ptr(rho),
                                                 _ptr(q), _ptr(o), _stream(stream)), "voldor_proposal_forward")
        return rho, q, o

    def proposal_train_step(self, net, flow, tnorm, idepth_t, rigid_t, mask, lam, lr, step, loss_out, stream=None):
        N, H, W, _ = flow.shape
        self._check(_LIB.voldor_proposal_train_step(
            self._h, ctypes.byref(self._net(net)), H, W, N, _ptr(flow), float(tnorm), _ptr(idepth_t), _ptr(rigid_t),
            _ptr(mask), float(lam), float(lr), int(step), _ptr(loss_out), _stream(stream)), "voldor_proposal_train_step")

    def conv3x3_bf16(self, x, w, bias=None, skip=None, stride=1, up=0, relu=0, want_y=True, stream=None):
        """x [H][W][Cin], w [Cout][3][3][Cin] as int16 tensors of BF16 bits -> (y bits, y FP32)."""
        H, W, Cin = x.shape
        Cout = w.shape[0]
        Hs, Ws = (2 * H, 2 * W) if up else (H, W)
        Ho, Wo = (Hs - 1) // stride + 1, (Ws - 1) // stride + 1
        y = torch.empty((Ho, Wo, Cout), dtype=torch.int16, device=x.device) if want_y else None
        yf = torch.empty((Ho, Wo, Cout), dtype=torch.float32, device=x.device)
        self._check(_LIB.voldor_conv3x3_bf16(self._h, H, W, Cin, Cout, stride, up, relu, _ptr(x), _ptr(w),
                                             _ptr(bias), _ptr(skip), _ptr(y), _ptr(yf), _stream(stream)),
                    "voldor_conv3x3_bf16")
        return y, yf

    def conv3x3_bf16_backward(self, x, w_t, dy, stride=1, up=0, stream=None):
        """-> (dx [H][W][Cin], dw [Cout][3][3][Cin], db [Cout]) FP32."""
        H, W, Cin = x.shape
        Cout = dy.shape[2]
        dx = torch.empty((H, W, Cin), dtype=torch.float32, device=x.device)
        dw = torch.empty((Cout, 3, 3, Cin), dtype=torch.float32, device=x.device)
        db = torch.empty(Cout, dtype=torch.float32, device=x.device)
        self._check(_LIB.voldor_conv3x3_bf16_backward(self._h, H, W, Cin, Cout, stride, up, _ptr(x), _ptr(w_t),
                                                      _ptr(dy), _ptr(dx), _ptr(dw), _ptr(db), _stream(stream)),
                    "voldor_conv3x3_bf16_backward")
        return dx, dw, db

    def align_p2p(self, ap, idepth1, idepth2, conf2, pose_inout, stream=None):
        """Returns (cov [n][36], stats [n][4], status [n]); pose_inout is updated in place."""
        n = idepth1.shape[0]
        dev = idepth1.device
        for t, dt in ((idepth1, torch.float32), (idepth2, torch.float32), (conf2, torch.float32),
                      (pose_inout, torch.float64)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise VoldorError("align inputs must be contiguous device tensors of the documented dtypes")
        if tuple(idepth1.shape) != (n, ap["H"], ap["W"]) or idepth2.shape != idepth1.shape \
                or conf2.shape != idepth1.shape or tuple(pose_inout.shape) != (n, 6):
            raise VoldorError("align input shapes disagree")
        a = AlignParams(**{k: ap[k] for k, _ in AlignParams._fields_})
        cov = torch.zeros((n, 36), dtype=torch.float64, device=dev)
        stats = torch.zeros((n, 4), dtype=torch.float64, device=dev)
        status = torch.zeros(n, dtype=torch.int32, device=dev)
        self._check(_LIB.voldor_align_p2p(self._h, ctypes.byref(a), n, _ptr(idepth1), _ptr(idepth2), _ptr(conf2),
                                          _ptr(pose_inout), _ptr(cov), _ptr(stats), _ptr(status),
                                          _stream(stream)), "voldor_align_p2p")
        return cov, stats, status

    def align_sim3(self, ap, idepth1, idepth2, conf2, pose_inout, scale_inout, stream=None):
        """7-DoF alignment: pose_inout [n][6] and scale_inout [n] (FP64 device tensors) are
        updated in place; returns (cov [n][49], stats [n][4], status [n])."""
        n = idepth1.shape[0]
        dev = idepth1.device
        for t, dt in ((idepth1, torch.float32), (idepth2, torch.float32), (conf2, torch.float32),
                      (pose_inout, torch.float64), (scale_inout, torch.float64)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise VoldorError("align inputs must be contiguous device tensors of the documented dtypes")
        if tuple(idepth1.shape) != (n, ap["H"], ap["W"]) or idepth2.shape != idepth1.shape \
                or conf2.shape != idepth1.shape or tuple(pose_inout.shape) != (n, 6) or tuple(scale_inout.shape) != (n,):
            raise VoldorError("align input shapes disagree")
        a = AlignParams(**{k: ap[k] for k, _ in AlignParams._fields_})
        cov = torch.zeros((n, 49), dtype=torch.float64, device=dev)
        stats = torch.zeros((n, 4), dtype=torch.float64, device=dev)
        status = torch.zeros(n, dtype=torch.int32, device=dev)
        self._check(_LIB.voldor_align_sim3(self._h, ctypes.byref(a), n, _ptr(idepth1), _ptr(idepth2), _ptr(conf2),
                                           _ptr(pose_inout), _ptr(scale_inout), _ptr(cov), _ptr(stats), _ptr(status),
                                           _stream(stream)), "voldor_align_sim3")
        return cov, stats, status

    def vc_scores(self, vp, idepth, conf, poses, tau, stream=None):
        """Visibility-coverage scores of frame 1's idepth [H][W] (conf [H][W] or None) against
        poses [n][6]: returns (out [n][5] FP64 device tensor, first index with VC < tau)."""
        dev = idepth.device
        poses = torch.as_tensor(poses, dtype=torch.float64).to(dev).reshape(-1, 6).contiguous()
        if idepth.dtype != torch.float32 or not idepth.is_cuda or not idepth.is_contiguous() \
                or tuple(idepth.shape) != (vp["H"], vp["W"]):
            raise VoldorError("idepth must be a contiguous FP32 [H][W] device tensor")
        if conf is not None and (conf.dtype != torch.float32 or conf.shape != idepth.shape or not conf.is_contiguous()):
            raise VoldorError("conf must be a contiguous FP32 [H][W] device tensor")
        n = poses.shape[0]
        out = torch.zeros((n, 5), dtype=torch.float64, device=dev)
        first = torch.zeros(1, dtype=torch.int32, device=dev)
        a = VcParams(**{k: vp[k] for k, _ in VcParams._fields_})
        self._check(_LIB.voldor_vc_scores(self._h, ctypes.byref(a), _ptr(idepth), _ptr(conf), n, _ptr(poses),
                                          float(tau), _ptr(out), _ptr(first), _stream(stream)), "voldor_vc_scores")
        return out, first
