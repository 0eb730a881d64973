"""Thin Python binding of the C ABI in ``include/hgs.h`` (ctypes).

Argument marshalling only: every stage of the cut and splatting path runs in
the HIP library ``libhgs.so``.  PyTorch provides device memory and the
stream.  Importing this module does not need a GPU; creating a
:class:`Renderer` does, and fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhgs.so")

OK, ERR_INVALID_ARG, ERR_OOM, ERR_HIP, ERR_STATE, ERR_CAPACITY = range(6)
_NAMES = {0: "HGS_OK", 1: "HGS_ERR_INVALID_ARG", 2: "HGS_ERR_OOM", 3: "HGS_ERR_HIP", 4: "HGS_ERR_STATE",
          5: "HGS_ERR_CAPACITY"}
EXPORTS = ("hgs_create", "hgs_destroy", "hgs_last_error", "hgs_set_stream", "hgs_upload", "hgs_bind_params",
           "hgs_build", "hgs_download", "hgs_cut", "hgs_cut_noalloc", "hgs_compact_mark", "hgs_compact_rebuild", "hgs_render", "hgs_last_render",
           "hgs_render_backward", "hgs_l1_loss", "hgs_stream_begin", "hgs_stream_end", "hgs_stream_cleanup",
           "hgs_stream_info", "hgs_adam_step", "hgs_backward_adam_step", "hgs_interior", "hgs_set_deterministic", "hgs_set_tuning", "hgs_get_buffer", "hgs_set_profiling",
           "hgs_kernel_time", "hgs_counters")
COUNTER_NAMES = ("cut", "visible", "pairs", "evaluated", "blended", "evaluated_t", "bwd_evaluated",
                 "bwd_evaluated_t", "bwd_contrib")
K_BLEND, K_BLEND_BWD, K_PREPROCESS_BWD = range(3)

(BUF_CUT_IDS, BUF_CUT_T, BUF_T_FINAL, BUF_N_LAST, BUF_N_BLEND, BUF_SGRAD, BUF_CUT_BASE, BUF_RANGES,
 BUF_VIS_RANK) = range(9)


class HgsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class LeavesDesc(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_int64), ("mean", ctypes.c_void_p), ("scale", ctypes.c_void_p),
                ("rot", ctypes.c_void_p), ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class HierarchyOut(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("parent", "child_begin", "child_count", "leaf_src", "bmin", "bmax",
                                               "mean", "scale", "rot", "opacity", "sh")]


class StreamStats(ctypes.Structure):
    _fields_ = [("cache_nodes", ctypes.c_int64), ("resident", ctypes.c_int64), ("frame", ctypes.c_int64),
                ("requested", ctypes.c_int64), ("transferred_total", ctypes.c_int64), ("overflow", ctypes.c_int32)]


class HierarchyDesc(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("sh_degree", ctypes.c_int32),
                ("parent", ctypes.c_void_p), ("child_begin", ctypes.c_void_p), ("child_count", ctypes.c_void_p),
                ("bmin", ctypes.c_void_p), ("bmax", ctypes.c_void_p), ("mean", ctypes.c_void_p),
                ("scale", ctypes.c_void_p), ("rot", ctypes.c_void_p), ("opacity", ctypes.c_void_p),
                ("sh", ctypes.c_void_p)]


class View(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("eye", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("z_near", ctypes.c_float),
                ("tau", ctypes.c_float)]


class Stats(ctypes.Structure):
    _fields_ = [("cut", ctypes.c_int64), ("visible", ctypes.c_int64), ("pairs", ctypes.c_int64),
                ("evaluated", ctypes.c_int64), ("blended", ctypes.c_int64), ("ms", ctypes.c_float * 8),
                ("render_id", ctypes.c_uint64)]

    def as_dict(self):
        return dict(cut=self.cut, visible=self.visible, pairs=self.pairs, evaluated=self.evaluated,
                    blended=self.blended, ms=list(self.ms), render_id=self.render_id)


class Adam(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p * 5), ("grad", ctypes.c_void_p * 5), ("m", ctypes.c_void_p * 5),
                ("v", ctypes.c_void_p * 5), ("lr", ctypes.c_float * 5), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("step", ctypes.c_int64)]


class Grads(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_void_p), ("scale", ctypes.c_void_p), ("rot", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("dt", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded ``libhgs.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2406_12080_amd.build` "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        P, c_int, vp = ctypes.POINTER, ctypes.c_int, ctypes.c_void_p
        L.hgs_create.argtypes = [P(vp), c_int, vp]
        L.hgs_destroy.argtypes = [vp]
        L.hgs_destroy.restype = None
        L.hgs_last_error.argtypes = [vp]
        L.hgs_last_error.restype = ctypes.c_char_p
        L.hgs_set_stream.argtypes = [vp, vp]
        L.hgs_upload.argtypes = [vp, P(HierarchyDesc), c_int]
        L.hgs_bind_params.argtypes = [vp, vp, vp, vp, vp, vp]
        L.hgs_build.argtypes = [vp, P(LeavesDesc), c_int, P(ctypes.c_int64)]
        L.hgs_download.argtypes = [vp, P(HierarchyOut), c_int]
        L.hgs_cut.argtypes = [vp, P(View), vp, vp, ctypes.c_int64, P(ctypes.c_int64)]
        L.hgs_cut_noalloc.argtypes = [vp, P(View), vp, vp, ctypes.c_int64, P(ctypes.c_int64)]
        L.hgs_compact_mark.argtypes = [vp, P(View), ctypes.c_int32, ctypes.c_float, ctypes.c_float, vp]
        L.hgs_compact_rebuild.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, vp, vp, P(ctypes.c_int64)]
        L.hgs_render.argtypes = [vp, P(View), ctypes.c_int32, P(vp), P(Stats)]
        L.hgs_last_render.argtypes = [vp, P(ctypes.c_uint64), P(ctypes.c_int32)]
        L.hgs_render_backward.argtypes = [vp, ctypes.c_uint64, ctypes.c_int32, P(vp), P(Grads)]
        L.hgs_l1_loss.argtypes = [vp, ctypes.c_uint64, ctypes.c_int32, P(vp), P(vp), vp]
        L.hgs_adam_step.argtypes = [vp, P(Adam)]
        L.hgs_backward_adam_step.argtypes = [vp, ctypes.c_uint64, ctypes.c_int32, P(vp), P(Adam)]
        L.hgs_stream_begin.argtypes = [vp, ctypes.c_int64]
        L.hgs_stream_end.argtypes = [vp]
        L.hgs_stream_cleanup.argtypes = [vp, ctypes.c_int32]
        L.hgs_stream_info.argtypes = [vp, P(StreamStats)]
        L.hgs_set_tuning.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.hgs_get_buffer.argtypes = [vp, ctypes.c_int32, P(vp), P(ctypes.c_int64)]
        L.hgs_interior.argtypes = [vp, vp, ctypes.c_int64, P(ctypes.c_int64)]
        L.hgs_set_deterministic.argtypes = [vp, ctypes.c_int32]
        L.hgs_set_profiling.argtypes = [vp, ctypes.c_int32]
        L.hgs_counters.argtypes = [vp, P(ctypes.c_int64), ctypes.c_int32]
        L.hgs_kernel_time.argtypes = [vp, ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_int64)]
        for f in EXPORTS:
            if f not in ("hgs_destroy", "hgs_last_error"):
                getattr(L, f).restype = c_int
        _lib = L
    return _lib


def make_view(v) -> View:
    """hgs_view from any object with R, eye, fx, fy, cx, cy, width, height,
    z_near, tau (e.g. ``synth.View``)."""
    out = View()
    R = np.asarray(v.R, np.float32).reshape(9)
    for k in range(9):
        out.R[k] = float(R[k])
    e = np.asarray(v.eye, np.float32).reshape(3)
    for k in range(3):
        out.eye[k] = float(e[k])
    out.fx, out.fy, out.cx, out.cy = float(v.fx), float(v.fy), float(v.cx), float(v.cy)
    out.width, out.height = int(v.width), int(v.height)
    out.z_near, out.tau = float(v.z_near), float(v.tau)
    return out


_hip = None


def _hip_memcpy_d2d(dst: int, src: int, nbytes: int) -> None:
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    r = _hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 3)  # device to device
    if r != 0:
        raise RuntimeError(f"hipMemcpy failed: {r}")


PARAM_FIELDS = ("mean", "scale", "rot", "opacity", "sh")


class Renderer:
    """One library context on one device (``hgs_create``)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._stream = stream
        self.L = lib()
        h = ctypes.c_void_p()
        st = self.L.hgs_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if st != OK:
            raise HgsError(st, "hgs_create failed")
        self.h = h
        self.n_nodes = 0
        self._keep = []
        self._last = None  # (render id, image shapes, cut size) of the last render

    def close(self):
        if getattr(self, "h", None):
            self.L.hgs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != OK:
            raise HgsError(st, self.L.hgs_last_error(self.h).decode())

    # -- hierarchy ---------------------------------------------------------
    def upload(self, hier) -> None:
        """Upload a hierarchy: a ``synth.Hierarchy``, or a dict of node-major
        arrays (see ``node_major``) as numpy arrays (host) or CUDA tensors
        (device)."""
        a = node_major(hier) if hasattr(hier, "arrays") else dict(hier)
        torch = self.torch
        on_dev = isinstance(a["mean"], torch.Tensor) and a["mean"].is_cuda
        keep = {}
        for k, dt in (("parent", np.int32), ("child_begin", np.int32), ("child_count", np.int32),
                      ("bmin", np.float32), ("bmax", np.float32), ("mean", np.float32), ("scale", np.float32),
                      ("rot", np.float32), ("opacity", np.float32), ("sh", np.float32)):
            x = a[k]
            if on_dev:
                x = x.contiguous()
                assert x.dtype == (torch.int32 if dt == np.int32 else torch.float32), k
                keep[k] = (x, x.data_ptr())
            else:
                x = np.ascontiguousarray(x, dt)
                keep[k] = (x, x.ctypes.data)
        d = HierarchyDesc()
        d.n_nodes = int(keep["parent"][0].shape[0])
        d.sh_degree = 3
        for k in keep:
            setattr(d, k, keep[k][1])
        self._check(self.L.hgs_upload(self.h, ctypes.byref(d), 1 if on_dev else 0))
        self.n_nodes = d.n_nodes

    def build(self, leaves) -> int:
        """Build the hierarchy over ``leaves`` on the device (``hgs_build``)
        and make it this renderer's.  ``leaves``: dict of node-major arrays
        pos or mean [n, 3], scale [n, 3], rot [n, 4], opacity [n], sh [n, 48]
        (numpy: host, CUDA tensors: device).  Returns the node count."""
        torch = self.torch
        a = dict(leaves)
        if "mean" not in a:
            a["mean"] = a["pos"]
        on_dev = isinstance(a["mean"], torch.Tensor) and a["mean"].is_cuda
        keep = {}
        for k in ("mean", "scale", "rot", "opacity", "sh"):
            x = a[k]
            if on_dev:
                x = x.contiguous()
                assert x.dtype == torch.float32, k
                keep[k] = (x, x.data_ptr())
            else:
                x = np.ascontiguousarray(x, np.float32)
                keep[k] = (x, x.ctypes.data)
        d = LeavesDesc()
        d.n_leaves = int(keep["opacity"][0].shape[0])
        for k in keep:
            setattr(d, k, keep[k][1])
        nn = ctypes.c_int64()
        self._check(self.L.hgs_build(self.h, ctypes.byref(d), 1 if on_dev else 0, ctypes.byref(nn)))
        self.n_nodes = int(nn.value)
        self._bound = None
        self._last = None
        return self.n_nodes

    def download(self, leaf_src: bool = False) -> dict:
        """The renderer's hierarchy as host numpy arrays in the hierarchy's
        storage layout (component-major, as ``synth.Hierarchy``): parent,
        child_begin, child_count (int32 [N]), bmin, bmax, mean, scale [3, N],
        rot [4, N], opacity [N], sh [48, N]; with ``leaf_src`` also the
        build's input index of every leaf node (-1 for interior nodes)."""
        N = self.n_nodes
        nm = dict(parent=np.zeros(N, np.int32), child_begin=np.zeros(N, np.int32),
                  child_count=np.zeros(N, np.int32), bmin=np.zeros((N, 3), np.float32),
                  bmax=np.zeros((N, 3), np.float32), mean=np.zeros((N, 3), np.float32),
                  scale=np.zeros((N, 3), np.float32), rot=np.zeros((N, 4), np.float32),
                  opacity=np.zeros(N, np.float32), sh=np.zeros((N, 48), np.float32))
        if leaf_src:
            nm["leaf_src"] = np.zeros(N, np.int32)
        o = HierarchyOut()
        for k, x in nm.items():
            setattr(o, k, x.ctypes.data)
        self._check(self.L.hgs_download(self.h, ctypes.byref(o), 0))
        out = {k: (np.ascontiguousarray(x.T) if x.ndim == 2 else x) for k, x in nm.items()}
        return out

    def bind(self, mean, scale, rot, opacity, sh) -> None:
        ts = (mean, scale, rot, opacity, sh)
        for t in ts:
            assert t.is_cuda and t.is_contiguous() and t.dtype == self.torch.float32
        self._bound = ts
        self._check(self.L.hgs_bind_params(self.h, *[ctypes.c_void_p(t.data_ptr()) for t in ts]))

    def unbind(self) -> None:
        self._bound = None
        self._check(self.L.hgs_bind_params(self.h, None, None, None, None, None))

    def set_tuning(self, tile_w: int, tile_h: int, batch: int = 0, persistent: int = 0) -> None:
        self._check(self.L.hgs_set_tuning(self.h, tile_w, tile_h, batch, int(persistent)))

    # -- cut -----------------------------------------------------------------
    def cut(self, view, capacity: int | None = None):
        torch = self.torch
        cap = capacity if capacity is not None else self.n_nodes
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        t = torch.empty(max(cap, 1), dtype=torch.float32, device=self.device)
        cnt = ctypes.c_int64()
        hv = make_view(view)
        self._check(self.L.hgs_cut(self.h, ctypes.byref(hv), ctypes.c_void_p(ids.data_ptr()),
                                   ctypes.c_void_p(t.data_ptr()), cap, ctypes.byref(cnt)))
        return ids[:cnt.value], t[:cnt.value]

    def cut_noalloc(self, view, ids, t=None) -> int:
        """``hgs_cut_noalloc`` into caller-given CUDA tensors (int32 ids,
        float32 t or None; capacity = len(ids)); returns the cut size."""
        assert ids.is_cuda and ids.dtype == self.torch.int32 and ids.is_contiguous()
        if t is not None:
            assert t.is_cuda and t.dtype == self.torch.float32 and t.numel() >= ids.numel()
        cnt = ctypes.c_int64()
        hv = make_view(view)
        self._check(self.L.hgs_cut_noalloc(self.h, ctypes.byref(hv), ctypes.c_void_p(ids.data_ptr()),
                                           ctypes.c_void_p(t.data_ptr() if t is not None else 0), ids.numel(),
                                           ctypes.byref(cnt)))
        return cnt.value

    def compact_mark(self, views, tau_min: float = 3.0, tau_max: float | None = None):
        """Keep flags of the hierarchy compaction (``hgs_compact_mark``) for
        these views: a bool CUDA tensor over the nodes.  ``tau_max`` defaults
        to half the largest image side."""
        torch = self.torch
        views = list(views)
        if tau_max is None:
            tau_max = 0.5 * max(max(v.width, v.height) for v in views)
        arr = (View * len(views))(*[make_view(v) for v in views])
        keep = torch.empty(max(self.n_nodes, 1), dtype=torch.uint8, device=self.device)
        self._check(self.L.hgs_compact_mark(self.h, arr, len(views), float(tau_min), float(tau_max),
                                            ctypes.c_void_p(keep.data_ptr())))
        return keep[:self.n_nodes].bool()

    # -- render ----------------------------------------------------------------
    def render(self, views, out=None, timed: bool = False):
        """Render a list of views; returns (images, stats dict).  ``out`` may
        hold preallocated float32 [H, W, 3] CUDA tensors."""
        torch = self.torch
        views = list(views)
        nv = len(views)
        arr = (View * nv)(*[make_view(v) for v in views])
        if out is None:
            out = [torch.empty((v.height, v.width, 3), dtype=torch.float32, device=self.device) for v in views]
        ptrs = (ctypes.c_void_p * nv)(*[o.data_ptr() for o in out])
        st = Stats()
        if timed:
            st.ms[0] = -1.0
        self._check(self.L.hgs_render(self.h, arr, nv, ptrs, ctypes.byref(st)))
        self._last_views = views
        self._last = (st.render_id, [(v.height, v.width, 3) for v in views], st.cut)
        return out, st.as_dict()

    def last_render(self):
        """(render id, view count) of the render whose state the context
        holds for the backward; (0, 0) when there is none."""
        rid, nv = ctypes.c_uint64(), ctypes.c_int32()
        self._check(self.L.hgs_last_render(self.h, ctypes.byref(rid), ctypes.byref(nv)))
        return rid.value, nv.value

    def backward(self, dL, grads: dict, dt=None, render_id: int | None = None) -> None:
        """Accumulate parameter gradients of a render into ``grads`` (dict of
        CUDA tensors keyed like the parameters).  ``render_id`` (default:
        this renderer's last render) names the render being differentiated;
        the library rejects it when a later render has replaced its state.
        ``dL`` holds one float32 [H, W, 3] CUDA tensor per view of that
        render; ``dt`` (optional) room for dL/dt of every cut entry."""
        torch = self.torch
        rid = self._check_cotangents(dL, render_id)
        if rid == self._last[0]:
            n_cut = self._last[2]
            if dt is not None and not (dt.is_cuda and dt.dtype == torch.float32 and dt.numel() >= n_cut):
                raise HgsError(ERR_INVALID_ARG, f"dt must be a float32 CUDA tensor of at least {n_cut} entries")
        comp = dict(mean=3, scale=3, rot=4, opacity=1, sh=48)
        for k in PARAM_FIELDS:
            t = grads[k]
            if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float32 and
                    t.numel() == comp[k] * self.n_nodes):
                raise HgsError(ERR_INVALID_ARG, f"grads[{k!r}] must be a contiguous float32 CUDA tensor of "
                                                f"{comp[k] * self.n_nodes} entries")
        dL = [g.contiguous() for g in dL]
        ptrs = (ctypes.c_void_p * len(dL))(*[g.data_ptr() for g in dL])
        g = Grads()
        for k in PARAM_FIELDS:
            setattr(g, k, grads[k].data_ptr())
        g.dt = dt.data_ptr() if dt is not None else None
        self._keep = dL
        self._check(self.L.hgs_render_backward(self.h, rid, len(dL), ptrs, ctypes.byref(g)))

    def _check_cotangents(self, dL, render_id):
        """The render id a backward names; checks the cotangents' shapes
        when it is this renderer's last render (the library rejects any
        other id)."""
        if self._last is None:
            raise HgsError(ERR_STATE, "no render on this renderer")
        rid = self._last[0] if render_id is None else int(render_id)
        if rid == self._last[0]:
            shapes = self._last[1]
            if len(dL) != len(shapes):
                raise HgsError(ERR_INVALID_ARG, f"{len(dL)} cotangents for a render of {len(shapes)} views")
            for k, (g, shp) in enumerate(zip(dL, shapes)):
                if not (g.is_cuda and g.dtype == self.torch.float32 and tuple(g.shape) == shp):
                    raise HgsError(ERR_INVALID_ARG, f"dL[{k}] must be a float32 CUDA tensor of shape {shp}, "
                                                    f"not {g.dtype} {tuple(g.shape)}")
        return rid

    def l1_loss(self, targets, dL=None, loss=None):
        """``hgs_l1_loss`` of this renderer's last render against ``targets``
        (one float32 [H, W, 3] CUDA tensor per view): writes the cotangent
        into ``dL`` (allocated when None) and the loss into ``loss`` (a
        float64 CUDA scalar, allocated when None); returns both.  Queued on
        the renderer's stream."""
        torch = self.torch
        if self._last is None:
            raise HgsError(ERR_STATE, "no render on this renderer")
        rid, shapes = self._last[0], self._last[1]
        if len(targets) != len(shapes):
            raise HgsError(ERR_INVALID_ARG, f"{len(targets)} targets for a render of {len(shapes)} views")
        if dL is None:
            dL = [torch.empty(shp, dtype=torch.float32, device=self.device) for shp in shapes]
        if loss is None:
            loss = torch.empty((), dtype=torch.float64, device=self.device)
        for k, (t, g, shp) in enumerate(zip(targets, dL, shapes)):
            for name, x in (("targets", t), ("dL", g)):
                if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and tuple(x.shape) == shp):
                    raise HgsError(ERR_INVALID_ARG, f"{name}[{k}] must be a contiguous float32 CUDA tensor of "
                                                    f"shape {shp}")
        assert loss.is_cuda and loss.dtype == torch.float64
        tp = (ctypes.c_void_p * len(targets))(*[t.data_ptr() for t in targets])
        gp = (ctypes.c_void_p * len(dL))(*[g.data_ptr() for g in dL])
        self._check(self.L.hgs_l1_loss(self.h, rid, len(dL), tp, gp, ctypes.c_void_p(loss.data_ptr())))
        return dL, loss

    # -- out-of-core rendering (hgs_stream_*) -------------------------------
    def stream_begin(self, cache_nodes: int) -> None:
        """Keep the parameters in pinned host memory and a device cache of
        ``cache_nodes`` records; renders transfer what their cuts need."""
        self._check(self.L.hgs_stream_begin(self.h, int(cache_nodes)))
        self._last = None

    def stream_end(self) -> None:
        self._check(self.L.hgs_stream_end(self.h))
        self._last = None

    def stream_cleanup(self, max_age: int) -> None:
        self._check(self.L.hgs_stream_cleanup(self.h, int(max_age)))

    def stream_info(self) -> dict:
        st = StreamStats()
        self._check(self.L.hgs_stream_info(self.h, ctypes.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in StreamStats._fields_}

    def set_deterministic(self, on: bool) -> None:
        """Deterministic-reduction mode of the backward (``hgs_set_deterministic``):
        no floating-point atomics, bit-identical gradients from run to run."""
        self._check(self.L.hgs_set_deterministic(self.h, 1 if on else 0))

    def n_interior(self) -> int:
        """Number of interior nodes of the current hierarchy (``hgs_interior``)."""
        n = ctypes.c_int64()
        self._check(self.L.hgs_interior(self.h, None, 0, ctypes.byref(n)))
        return int(n.value)

    def interior_ids(self):
        """The interior node ids in ascending order (int32 CUDA tensor): the
        row order of the optimiser moments."""
        torch = self.torch
        n = self.n_interior()
        out = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)[:n]
        cnt = ctypes.c_int64()
        self._check(self.L.hgs_interior(self.h, ctypes.c_void_p(out.data_ptr()), n, ctypes.byref(cnt)))
        return out

    def adam_moments(self, params: dict) -> tuple:
        """Zeroed first and second moments for ``adam_step``: per parameter
        group an [n_interior, components] float32 CUDA tensor."""
        torch = self.torch
        n = self.n_interior()
        m, v = {}, {}
        for k, t in params.items():
            comp = t.numel() // max(t.shape[0], 1) if t.dim() > 1 else 1
            m[k] = torch.zeros((n, comp), dtype=torch.float32, device=t.device)
            v[k] = torch.zeros((n, comp), dtype=torch.float32, device=t.device)
        return m, v

    def adam_step(self, params: dict, grads: dict, m: dict, v: dict, lr, step: int, beta1: float = 0.9,
                  beta2: float = 0.999, eps: float = 1e-15) -> None:
        """One optimiser step on the interior nodes (``hgs_adam_step``); all
        dicts hold CUDA tensors keyed like the parameters, ``m`` and ``v``
        with one row per interior node (``adam_moments``); ``lr`` is one
        float or a dict per parameter group.  Zeroes ``grads``."""
        a = self._adam_args(params, grads, m, v, lr, step, beta1, beta2, eps)
        self._check(self.L.hgs_adam_step(self.h, ctypes.byref(a)))

    def _adam_args(self, params, grads, m, v, lr, step, beta1, beta2, eps):
        a = Adam()
        comp = dict(mean=3, scale=3, rot=4, opacity=1, sh=48)
        n_int = self.n_interior()
        for k, name in enumerate(PARAM_FIELDS):
            for arr, d, rows in ((a.param, params, self.n_nodes), (a.grad, grads, self.n_nodes), (a.m, m, n_int),
                                 (a.v, v, n_int)):
                if d is None:
                    continue
                t = d[name]
                if not (t.is_cuda and t.is_contiguous() and t.dtype == self.torch.float32 and
                        t.numel() == comp[name] * rows):
                    raise HgsError(ERR_INVALID_ARG, f"{name}: optimiser arrays must be contiguous float32 CUDA "
                                                    f"tensors of {rows} x {comp[name]} entries")
                arr[k] = t.data_ptr()
            a.lr[k] = float(lr[name] if isinstance(lr, dict) else lr)
        a.beta1, a.beta2, a.eps, a.step = float(beta1), float(beta2), float(eps), int(step)
        return a

    def backward_adam_step(self, dL, params: dict, m: dict, v: dict, lr, step: int, beta1: float = 0.9,
                           beta2: float = 0.999, eps: float = 1e-15, render_id: int | None = None) -> None:
        """The backward of a render with the optimiser step applied in the
        gradient gather (``hgs_backward_adam_step``): the result of
        ``backward`` into zeroed gradients followed by ``adam_step``, with no
        gradient arrays.  Arguments as for those two calls."""
        rid = self._check_cotangents(dL, render_id)
        dL = [g.contiguous() for g in dL]
        ptrs = (ctypes.c_void_p * len(dL))(*[g.data_ptr() for g in dL])
        a = self._adam_args(params, None, m, v, lr, step, beta1, beta2, eps)
        self._keep = dL
        self._check(self.L.hgs_backward_adam_step(self.h, rid, len(dL), ptrs, ctypes.byref(a)))

    def counters(self) -> dict:
        out = (ctypes.c_int64 * len(COUNTER_NAMES))()
        self._check(self.L.hgs_counters(self.h, out, len(COUNTER_NAMES)))
        return dict(zip(COUNTER_NAMES, list(out)))

    def set_profiling(self, on: bool) -> None:
        self._check(self.L.hgs_set_profiling(self.h, 1 if on else 0))

    def kernel_time(self, which: int):
        """(total milliseconds, launches) of kernel `which` since profiling was switched on."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.L.hgs_kernel_time(self.h, which, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def buffer(self, which: int, dtype):
        """Copy of an internal buffer of the last render (see hgs_get_buffer)."""
        torch = self.torch
        p = ctypes.c_void_p()
        n = ctypes.c_int64()
        self._check(self.L.hgs_get_buffer(self.h, which, ctypes.byref(p), ctypes.byref(n)))
        out = torch.empty(max(n.value, 1), dtype=dtype, device=self.device)
        torch.cuda.synchronize(self.device)
        if n.value:
            _hip_memcpy_d2d(out.data_ptr(), p.value, n.value * out.element_size())
        return out[:n.value]


NODE_MAJOR_FIELDS = ("bmin", "bmax", "mean", "scale", "rot", "sh")


def node_major(hier) -> dict:
    """The arrays of a ``synth.Hierarchy`` (component-major, [k][N]) in the
    C ABI's node-major layout ([N][k]: a node's components contiguous)."""
    a = dict(hier.arrays())
    for k in NODE_MAJOR_FIELDS:
        a[k] = np.ascontiguousarray(np.asarray(a[k]).T)
    return a


def params_to_device(hier, device="cuda"):
    """The five parameter arrays of a hierarchy (a ``synth.Hierarchy`` or a
    node-major dict) as contiguous CUDA tensors in the node-major layout."""
    import torch
    a = node_major(hier) if hasattr(hier, "arrays") else hier
    return {k: torch.as_tensor(np.ascontiguousarray(a[k], np.float32)).to(device) for k in PARAM_FIELDS}
