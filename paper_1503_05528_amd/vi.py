"""ctypes binding of libvi (include/vi.h): argument marshalling only.

Device buffers are torch tensors on the GPU; every step of the method runs
in libvi's HIP kernels.  Loading fails loudly when libvi.so is missing: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvi.so")

WEIGHTED, MEAN, BEST = 0, 1, 2
STATUS = {0: "VI_OK", -1: "VI_E_INVAL", -2: "VI_E_NOMEM", -3: "VI_E_HIP", -4: "VI_E_STATE",
          -5: "VI_E_EMPTY_SOURCE", -6: "VI_E_BUDGET"}

_LIB = None


class Params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32),
        ("patch", C.c_int32 * 3),
        ("levels", C.c_int32),
        ("lambda_", C.c_int32),
        ("pm_iters", C.c_int32),
        ("n_jf", C.c_int32),
        ("jf_steps", C.c_int32 * 8),
        ("rho", C.c_double),
        ("em_max_iters", C.c_int32),
        ("em_tol", C.c_double),
        ("recon_mode", C.c_int32),
        ("seed", C.c_uint64),
        ("temporal_subsample", C.c_int32),
        ("reduce_dims", C.c_int32),
        ("wide_pass_max", C.c_int32),
    ]


class ViError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {msg}")
        self.status = status


# exported symbols and their (restype, argtypes)
_vp, _i32, _i64, _u64, _f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
class AlignParams(C.Structure):
    _fields_ = [("levels", C.c_int32), ("iters", C.c_int32), ("tukey_c", C.c_double)]


_f64p = C.POINTER(C.c_double)

SIGNATURES = {
    "vi_align_params_default": (_i32, [C.POINTER(AlignParams)]),
    "vi_align_estimate": (_i32, [_vp, _vp, _i32, _i32, _i32, C.POINTER(AlignParams), _f64p,
                                 _vp]),
    "vi_align_compose": (_i32, [_f64p, _i32, _f64p]),
    "vi_align_warp": (_i32, [_vp, _vp, _i32, _i32, _i32, _f64p, _vp, _vp, _vp]),
    "vi_align_unwarp": (_i32, [_vp, _vp, _vp, _i32, _i32, _i32, _f64p, _vp, _vp]),
    "vi_set_reduction": (_i32, [_vp, _i32, C.POINTER(C.c_int16), _i32]),
    "vi_features": (_i32, [_vp, _i32, _i32, _vp]),
    "vi_pca_moments": (_i32, [_vp, _i32, _i32, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                              C.POINTER(_i64)]),
    "vi_pca_basis": (_i32, [_vp, _i32, _i32, _i32, _i32, C.POINTER(C.c_int16), _f64p]),
    "vi_closer_than_constant": (_i32, [_vp, _i32, _vp, _i32, _i32, _i32, _i32, _i32, _i32,
                                       _i32, _vp, _vp]),
    "vi_params_default": (_i32, [C.c_void_p]),
    "vi_debug_fail_allocs": (_i64, [_i64]),
    "vi_create": (_i32, [C.POINTER(_vp), C.c_void_p, _i32, _i32, _i32, _vp, _vp, _vp]),
    "vi_level_info": (_i32, [_vp, _i32, C.POINTER(_i32), C.POINTER(_i64)]),
    "vi_level_sets": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "vi_nnf_search": (_i32, [_vp, _i32, _i32]),
    "vi_reconstruct": (_i32, [_vp, _i32, _i32, _vp, _vp]),
    "vi_inpaint_level": (_i32, [_vp, _i32, C.POINTER(_i32)]),
    "vi_onion_init": (_i32, [_vp, C.POINTER(_i32)]),
    "vi_onion_layer": (_i32, [_vp, _vp, _i32, _vp, C.POINTER(C.c_int64)]),
    "vi_onion_layer_noalloc": (_i32, [_vp, _vp, _i32, _vp, C.POINTER(C.c_int64)]),
    "vi_transition": (_i32, [_vp, _i32]),
    "vi_inpaint": (_i32, [_vp, _vp]),
    "vi_get_state": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "vi_set_state": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "vi_footprint_bytes": (C.c_size_t, [C.c_void_p, _i32, _i32, _i32, _f64]),
    "vi_ctx_bytes": (C.c_size_t, [_vp]),
    "vi_pool_trim": (C.c_size_t, []),
    "vi_set_stream": (_i32, [_vp, _vp]),
    "vi_destroy": (None, [_vp]),
    "vi_last_error": (C.c_char_p, []),
    "vi_nominal_evals": (_i64, [_vp, _i32]),
    "vi_get_counters": (_i32, [_vp, _vp]),
    "vi_reset_counters": (_i32, [_vp]),
    "vi_profile": (_i32, [_vp, _i32]),
    "vi_profile_read": (_i32, [_vp, _vp, _i32]),
    "vi_output": (_i32, [_vp, _vp]),
    "vi_done": (_i32, [_vp]),
    "vi_batch_create": (_i32, [C.POINTER(_vp), _vp, _vp]),
    "vi_batch_add": (_i32, [_vp, _vp]),
    "vi_batch_remove": (_i32, [_vp, _vp]),
    "vi_batch_step": (_i32, [_vp, C.POINTER(_i32)]),
    "vi_batch_get_tune": (_i32, [_vp, _vp]),
    "vi_batch_size": (_i32, [_vp]),
    "vi_batch_destroy": (None, [_vp]),
}


class Tune(C.Structure):
    _fields_ = [("block", C.c_int32), ("grid_mult", C.c_int32), ("tuned", C.c_int32)]


class Counters(C.Structure):
    _fields_ = [("nominal_evals", C.c_int64), ("effective_evals", C.c_int64),
                ("searches", C.c_int64), ("em_iters", C.c_int64), ("recon_pixels", C.c_int64),
                ("pass_evals", C.c_int64), ("init_evals", C.c_int64),
                ("onion_evals", C.c_int64), ("pass_wide_evals", C.c_int64)]


class KernelTime(C.Structure):
    _fields_ = [("kind", C.c_int32), ("level", C.c_int32), ("units", C.c_int64),
                ("ms", C.c_float), ("launches", C.c_int32)]


KERNEL_KINDS = {0: "init", 1: "pass", 2: "recon", 3: "other", 4: "onion", 5: "pass_wide"}


def lib():
    """Loads libvi.so (built by paper_1503_05528_amd/build.py)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libvi.so not found at {LIB_PATH}: build it with "
                               "`python paper_1503_05528_amd/build.py`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _check(fn, st):
    if st != 0:
        raise ViError(fn, st, lib().vi_last_error().decode())


def default_params(**kw) -> Params:
    p = Params()
    _check("vi_params_default", lib().vi_params_default(C.byref(p)))
    for k, v in kw.items():
        if k == "jf_steps":
            p.n_jf = len(v)
            for i, s in enumerate(v):
                p.jf_steps[i] = s
        elif k == "patch":
            for i, s in enumerate(v):
                p.patch[i] = s
        elif k == "lam":
            p.lambda_ = v
        else:
            setattr(p, k, v)
    return p


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def footprint_bytes(params: Params, W, H, T, hole_fraction) -> int:
    return int(lib().vi_footprint_bytes(C.byref(params), W, H, T, float(hole_fraction)))


def pool_trim() -> int:
    """Frees the device memory libvi keeps from destroyed contexts (current
    device); returns the bytes freed."""
    return int(lib().vi_pool_trim())


def fail_allocs(n: int) -> int:
    """Failure injection for tests: the next n context allocations succeed,
    later ones fail (n < 0: off).  Returns the pool bytes held by live
    contexts."""
    return int(lib().vi_debug_fail_allocs(int(n)))


class Clip:
    """One clip's device state in libvi.

    video: uint8 tensor [T][H][W][3] on the GPU; mask: uint8 [T][H][W]."""

    def __init__(self, video: torch.Tensor, mask: torch.Tensor, params: Params | None = None,
                 stream: torch.cuda.Stream | None = None, **kw):
        self.params = params if params is not None else default_params(**kw)
        assert video.dtype == torch.uint8 and mask.dtype == torch.uint8
        T, H, W, ch = video.shape
        assert ch == 3 and tuple(mask.shape) == (T, H, W)
        self.W, self.H, self.T = W, H, T
        self.device = video.device
        self.stream = stream
        video = video.contiguous()
        mask = mask.contiguous()
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib().vi_create(C.byref(h), C.byref(self.params), W, H, T, _ptr(video),
                                 _ptr(mask), _stream_handle(stream))
        _check("vi_create", st)
        self.h = h
        self._abs = torch.zeros(1, dtype=torch.int64, device=self.device)
        # set when the clip joins a batch: its work then runs on the batch's
        # stream, so tensor results are synchronised before they are returned
        self._foreign_stream = False

    def close(self):
        if getattr(self, "h", None):
            lib().vi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self.stream = stream
        _check("vi_set_stream", lib().vi_set_stream(self.h, _stream_handle(stream)))

    @property
    def levels(self):
        return self.params.levels

    def info(self, level):
        d = (C.c_int32 * 3)()
        c = (C.c_int64 * 3)()
        _check("vi_level_info", lib().vi_level_info(self.h, level, d, c))
        return tuple(d), tuple(c)

    def dims(self, level):
        return self.info(level)[0]

    def nbytes(self):
        return int(lib().vi_ctx_bytes(self.h))

    def _new(self, shape, dtype):
        return torch.empty(shape, dtype=dtype, device=self.device)

    def _settle(self):
        if self._foreign_stream:
            torch.cuda.synchronize(self.device)

    def sets(self, level):
        W, H, T = self.dims(level)
        hole, dsrc, htil = (self._new((T, H, W), torch.uint8) for _ in range(3))
        _check("vi_level_sets", lib().vi_level_sets(self.h, level, _ptr(hole), _ptr(dsrc),
                                                    _ptr(htil)))
        self._settle()
        return hole, dsrc, htil

    def get_state(self, level):
        W, H, T = self.dims(level)
        rgbt = self._new((T, H, W, 5), torch.uint8)
        cand = self._new((T, H, W), torch.int32)
        dist = self._new((T, H, W), torch.int32)
        nvox = self._new((T, H, W), torch.uint8)
        _check("vi_get_state", lib().vi_get_state(self.h, level, _ptr(rgbt), _ptr(cand),
                                                  _ptr(dist), _ptr(nvox)))
        self._settle()
        return rgbt, cand, dist, nvox

    def set_state(self, level, rgbt=None, cand=None, dist=None, nvox=None):
        def dev(a, dt):
            if a is None:
                return None
            t = torch.as_tensor(a)
            return t.to(device=self.device, dtype=dt).contiguous()
        rgbt, cand, dist, nvox = (dev(rgbt, torch.uint8), dev(cand, torch.int32),
                                  dev(dist, torch.int32), dev(nvox, torch.uint8))
        _check("vi_set_state", lib().vi_set_state(self.h, level, _ptr(rgbt), _ptr(cand),
                                                  _ptr(dist), _ptr(nvox)))

    def nnf_search(self, level, em_iter=0):
        _check("vi_nnf_search", lib().vi_nnf_search(self.h, level, em_iter))

    def reconstruct(self, level, mode=WEIGHTED, want_out=True):
        (_, _, _), (nH, _, _) = self.info(level)
        out = self._new((nH, 5), torch.float32) if want_out else None
        _check("vi_reconstruct", lib().vi_reconstruct(self.h, level, mode, _ptr(out),
                                                      _ptr(self._abs)))
        self._settle()
        return out, self._abs

    def inpaint_level(self, level):
        k = C.c_int32(0)
        _check("vi_inpaint_level", lib().vi_inpaint_level(self.h, level, C.byref(k)))
        return int(k.value)

    def onion_init(self):
        k = C.c_int32(0)
        _check("vi_onion_init", lib().vi_onion_init(self.h, C.byref(k)))
        return int(k.value)

    def onion_layer(self, Hp, layer, out=None, noalloc=False):
        """One onion-peel layer: Hp (device uint8 [T][H][W] of the coarsest
        level) is replaced by its erosion; returns the layer's reconstructed
        values [|layer|][5] in [0,1].  out: a float32 device buffer of at
        least |layer| rows to write them to (else one is allocated);
        noalloc: the variant whose work buffers are the library's fixed
        scratch (vi_onion_layer_noalloc)."""
        if out is None:
            nb = int(torch.count_nonzero(Hp))
            out = self._new((max(nb, 1), 5), torch.float32)
        n = C.c_int64(0)
        name = "vi_onion_layer_noalloc" if noalloc else "vi_onion_layer"
        _check(name, getattr(lib(), name)(self.h, _ptr(Hp), layer, _ptr(out), C.byref(n)))
        return out[:int(n.value)]

    def transition(self, level):
        _check("vi_transition", lib().vi_transition(self.h, level))

    # ------------------------------------------- reduced patch space (Sec. 5)
    @property
    def patch_dim(self):
        return 5 * self.params.patch[0] * self.params.patch[1] * self.params.patch[2]

    def pca_moments(self, level, n_max=65536):
        """(S1 [dim], S2 [dim][dim], n): exact moments of the sampled source
        patch vectors (host arrays)."""
        import numpy as np
        dim = self.patch_dim
        S1 = np.zeros(dim, np.uint64)
        S2 = np.zeros((dim, dim), np.uint64)
        n = C.c_int64(0)
        _check("vi_pca_moments", lib().vi_pca_moments(
            self.h, level, n_max, S1.ctypes.data_as(C.POINTER(C.c_uint64)),
            S2.ctypes.data_as(C.POINTER(C.c_uint64)), C.byref(n)))
        return S1, S2, int(n.value)

    def pca_basis(self, level, d, n_max=65536, iters=64):
        """(Q [d][dim] int16, captured variance [d]) of the level's source
        patches, computed on the GPU."""
        import numpy as np
        Q = np.zeros((d, self.patch_dim), np.int16)
        var = np.zeros(d, np.float64)
        _check("vi_pca_basis", lib().vi_pca_basis(
            self.h, level, d, n_max, iters, Q.ctypes.data_as(C.POINTER(C.c_int16)),
            var.ctypes.data_as(_f64p)))
        return Q, var

    def set_reduction(self, level, Q):
        """The level's searches compare the features of basis Q [d][dim]
        (host int16 array; None: the exact distance again)."""
        import numpy as np
        if Q is None:
            _check("vi_set_reduction", lib().vi_set_reduction(self.h, level, None, 0))
            return
        q = np.ascontiguousarray(Q, np.int16)
        _check("vi_set_reduction", lib().vi_set_reduction(
            self.h, level, q.ctypes.data_as(C.POINTER(C.c_int16)), q.shape[0]))

    def features(self, level, d):
        """The level's voxel features, device int32 [T][H][W][d]."""
        W, H, T = self.dims(level)
        out = self._new((T, H, W, d), torch.int32)
        _check("vi_features", lib().vi_features(self.h, level, d, _ptr(out)))
        return out

    def inpaint(self, out: torch.Tensor | None = None):
        if out is None:
            out = self._new((self.T, self.H, self.W, 3), torch.uint8)
        _check("vi_inpaint", lib().vi_inpaint(self.h, _ptr(out)))
        return out

    def done(self) -> bool:
        return bool(lib().vi_done(self.h))

    def output(self, out: torch.Tensor | None = None):
        if out is None:
            out = self._new((self.T, self.H, self.W, 3), torch.uint8)
        _check("vi_output", lib().vi_output(self.h, _ptr(out)))
        return out

    def nominal_evals(self, level):
        return int(lib().vi_nominal_evals(self.h, level))

    def counters(self) -> dict:
        c = Counters()
        _check("vi_get_counters", lib().vi_get_counters(self.h, C.byref(c)))
        return {k: int(getattr(c, k)) for k, _ in Counters._fields_}

    def reset_counters(self):
        _check("vi_reset_counters", lib().vi_reset_counters(self.h))

    def profile(self, on: bool = True, kinds=None):
        """Times launches with events: all kinds, or those named in kinds
        (e.g. ("pass",)); on=False stops."""
        mask = 0
        if on:
            names = kinds if kinds is not None else KERNEL_KINDS.values()
            for k, name in KERNEL_KINDS.items():
                if name in names:
                    mask |= 1 << k
        _check("vi_profile", lib().vi_profile(self.h, mask))

    def profile_read(self, cap: int = 1 << 16):
        buf = (KernelTime * cap)()
        n = lib().vi_profile_read(self.h, buf, cap)
        if n < 0:
            _check("vi_profile_read", n)
        return [(KERNEL_KINDS[buf[i].kind], buf[i].level, int(buf[i].units), float(buf[i].ms),
                 int(buf[i].launches)) for i in range(n)]


class Batch:
    """Clips that advance together, one EM iteration per step, each step one
    captured graph launch over all members (vi_batch_*).

    tune: None to autotune at the first step, or (block, grid_mult)."""

    def __init__(self, tune=None, stream: torch.cuda.Stream | None = None):
        h = C.c_void_p()
        t = None
        if tune is not None:
            t = Tune(int(tune[0]), int(tune[1]), 1)
        sh = C.c_void_p(stream.cuda_stream) if stream is not None else None
        _check("vi_batch_create", lib().vi_batch_create(C.byref(h),
                                                        C.byref(t) if t is not None else None, sh))
        self.h = h
        self.members = []

    def close(self):
        if getattr(self, "h", None):
            lib().vi_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, clip: "Clip"):
        torch.cuda.synchronize(clip.device)  # inputs written on torch's stream
        _check("vi_batch_add", lib().vi_batch_add(self.h, clip.h))
        clip._foreign_stream = True
        self.members.append(clip)

    def remove(self, clip: "Clip"):
        _check("vi_batch_remove", lib().vi_batch_remove(self.h, clip.h))
        self.members.remove(clip)

    def step(self) -> int:
        n = C.c_int32(0)
        _check("vi_batch_step", lib().vi_batch_step(self.h, C.byref(n)))
        return int(n.value)

    def tune(self):
        t = Tune()
        _check("vi_batch_get_tune", lib().vi_batch_get_tune(self.h, C.byref(t)))
        return (t.block, t.grid_mult) if t.tuned else None

    def __len__(self):
        return int(lib().vi_batch_size(self.h))

    def run(self, max_steps: int = 100000) -> int:
        """Steps until every member has finished; returns the step count."""
        for k in range(max_steps):
            if self.step() == len(self.members):
                return k + 1
        raise RuntimeError("batch did not finish")



# ---------------------------------------------------------------- realignment
# (Sec. 3.4, Alg. 2, and the inverse warp of Alg. 4)

def align_params(**kw) -> AlignParams:
    p = AlignParams()
    _check("vi_align_params_default", lib().vi_align_params_default(C.byref(p)))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _f64(a):
    import numpy as np
    a = np.ascontiguousarray(a, np.float64)
    return a, a.ctypes.data_as(_f64p)


def align_estimate(video: torch.Tensor, mask: torch.Tensor, stream=None, **kw):
    """theta [T-1][6] (numpy float64): the dominant affine motion of every
    pair of successive frames; video [T][H][W][3] and mask [T][H][W] uint8 on
    the GPU."""
    import numpy as np
    T, H, W, _ = video.shape
    th = np.zeros((T - 1, 6), np.float64)
    p = align_params(**kw)
    torch.cuda.synchronize(video.device)
    _check("vi_align_estimate", lib().vi_align_estimate(
        _ptr(video), _ptr(mask), W, H, T, C.byref(p), th.ctypes.data_as(_f64p),
        _stream_handle(stream)))
    return th


def align_compose(theta, T: int):
    """M [T][6]: every frame's map to the reference (middle) frame."""
    import numpy as np
    th, thp = _f64(theta)
    M = np.zeros((T, 6), np.float64)
    _check("vi_align_compose", lib().vi_align_compose(thp, T, M.ctypes.data_as(_f64p)))
    return M


def align_warp(video: torch.Tensor, mask: torch.Tensor, M, stream=None):
    """The aligned video and occlusion (device tensors)."""
    T, H, W, _ = video.shape
    out = torch.empty_like(video)
    om = torch.empty_like(mask)
    Mm, Mp = _f64(M)
    torch.cuda.synchronize(video.device)
    _check("vi_align_warp", lib().vi_align_warp(_ptr(video), _ptr(mask), W, H, T, Mp, _ptr(out),
                                                _ptr(om), _stream_handle(stream)))
    return out, om


def align_unwarp(aligned: torch.Tensor, video: torch.Tensor, mask: torch.Tensor, M,
                 stream=None):
    """The input video with its occluded pixels taken from the aligned
    (inpainted) video at their reference positions (device tensor)."""
    T, H, W, _ = video.shape
    out = torch.empty_like(video)
    Mm, Mp = _f64(M)
    torch.cuda.synchronize(video.device)
    _check("vi_align_unwarp", lib().vi_align_unwarp(_ptr(aligned), _ptr(video), _ptr(mask), W,
                                                    H, T, Mp, _ptr(out),
                                                    _stream_handle(stream)))
    return out


def inpaint_realigned(video: torch.Tensor, mask: torch.Tensor, align=None, **kw):
    """Alg. 4 with its realignment: estimate, compose, warp, inpaint the
    aligned video, unwarp into the original occlusion.  Returns (output,
    theta, M)."""
    T = video.shape[0]
    theta = align_estimate(video, mask, **(align or {}))
    M = align_compose(theta, T)
    av, am = align_warp(video, mask, M)
    g = Clip(av, am, **kw)
    inp = g.inpaint()
    g.close()
    return align_unwarp(inp, video, mask, M), theta, M


def closer_than_constant(ref: torch.Tensor, vol: torch.Tensor, patch, mu: int = 128,
                         out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """The textured-patch count of App. B on the GPU: out[r] = the number of
    patches V of the grey volume ``vol`` [T][H][W] (uint8, device) with
    SSD(ref[r], V) < SSD(ref[r], Z), Z the constant patch of value ``mu``.
    ``ref`` is [n][pt][ph][pw] (or [n][pw*ph*pt]) uint8 on the device and
    ``patch`` = (pw, ph, pt).  Returns int64 counts (device); runs on
    ``stream`` (default: the current stream) and synchronises it."""
    pw, ph, pt = (int(v) for v in patch)
    n = ref.shape[0]
    if ref.numel() != n * pw * ph * pt:
        raise ValueError("ref must hold n patches of pw * ph * pt voxels")
    T, H, W = vol.shape
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=vol.device)
    _check("vi_closer_than_constant", lib().vi_closer_than_constant(
        _ptr(ref) if n else None, n, _ptr(vol), W, H, T, pw, ph, pt, int(mu),
        _ptr(out) if n else None, _stream_handle(stream)))
    return out
