"""Python binding of libtoi (argument marshalling only).

Every step of the imaging path runs in the HIP library; this module turns
torch device tensors into the pointers and sizes of the C ABI declared in
``include/toi.h`` and raises on any non-OK status.  It never falls back to
another implementation: without the built library (``libtoi.so`` next to
this file) or without a GPU every call fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtoi.so")

TOI_OK, TOI_EINVAL, TOI_ENOMEM, TOI_EDEVICE, TOI_EUNSUPPORTED = range(5)
STATUS_NO_SAMPLES, STATUS_DEGENERATE, STATUS_PLANES, STATUS_OVERFLOW = 1, 2, 4, 8
INPUT_FLAG, INPUT_WEIGHT, INPUT_GAINS = 1, 2, 4


class ToiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libtoi error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("n_pix", ctypes.c_int32), ("cell_deg", ctypes.c_double), ("mode", ctypes.c_int32),
        ("n_slab", ctypes.c_int32), ("cheb_k", ctypes.c_int32), ("alpha_target", ctypes.c_double),
        ("cheb_gamma", ctypes.c_double), ("max_planes", ctypes.c_int32), ("support", ctypes.c_int32),
        ("corr_mask", ctypes.c_uint32), ("tile", ctypes.c_int32), ("n_row_max", ctypes.c_int32),
        ("n_chan", ctypes.c_int32), ("n_corr", ctypes.c_int32), ("n_ant", ctypes.c_int32),
        ("bin_cap", ctypes.c_int32),
    ]


class Snapshot(ctypes.Structure):
    _fields_ = [
        ("uvw", ctypes.c_void_p), ("vis", ctypes.c_void_p), ("flag", ctypes.c_void_p),
        ("weight", ctypes.c_void_p), ("freq", ctypes.c_void_p), ("ant1", ctypes.c_void_p),
        ("ant2", ctypes.c_void_p), ("gains", ctypes.c_void_p), ("n_row", ctypes.c_int32),
    ]


_lib = None

# exported functions and their C signatures
_SIGS = {
    "toi_params_default": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_double,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "toi_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "toi_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "toi_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "toi_grid": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Snapshot)]),
    "toi_image": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "toi_degrid": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Snapshot),
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "fitrig_tlisi": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4),
    "fitrig_tlisi_noalloc": (ctypes.c_int, [ctypes.c_void_p] * 3 + [ctypes.c_int32, ctypes.c_int32,
                                                                    ctypes.c_void_p, ctypes.c_void_p]),
    "fitrig_detect": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_int32, ctypes.c_void_p]),
    "fitrig_detect_cube": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "fitrig_localise": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                       ctypes.c_void_p]),
    "fitrig_strongest_map": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_int32, ctypes.c_void_p]),
    "toi_image_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Snapshot), ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "toi_ingest": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Snapshot), ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "toi_batch_inputs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32,
                                        ctypes.POINTER(Snapshot)]),
    "toi_batch_fill": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Snapshot)]),
    "toi_batch_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64)]),
    "toi_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_uint32)]),
    "toi_bin_info": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 4),
    "toi_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "toi_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "toi_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Snapshot), ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_float)]),
    "toi_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "toi_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
}

TUNE_VARIANTS = 12

STAGES = ("prep", "bin", "grid", "fft_rows", "fft_cols", "reproject", "tlisi", "degrid", "batch", "detect")


def lib():
    """Load libtoi.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2512_06254_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(code, ctx=None):
    if code != TOI_OK:
        msg = lib().toi_last_error(ctx)
        raise ToiError(code, msg.decode() if msg else "")


def snapshot_struct(snap: dict, device=None) -> Snapshot:
    """Descriptor of a snapshot whose arrays are torch tensors on the GPU."""
    import torch
    need = {"uvw": torch.float64, "vis": torch.complex64, "freq": torch.float64}
    opt = {"flag": torch.uint8, "weight": torch.float32, "ant1": torch.int32, "ant2": torch.int32,
           "gains": torch.complex64}
    for k, dt in list(need.items()) + list(opt.items()):
        t = snap.get(k)
        if t is None:
            if k in need and snap["uvw"].shape[0] > 0:
                raise ValueError(f"snapshot is missing {k}")
            continue
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise TypeError(f"snapshot[{k!r}] must be a contiguous {dt} CUDA tensor")
    return Snapshot(uvw=_ptr(snap["uvw"]), vis=_ptr(snap["vis"]), flag=_ptr(snap.get("flag")),
                    weight=_ptr(snap.get("weight")), freq=_ptr(snap["freq"]),
                    ant1=_ptr(snap.get("ant1")), ant2=_ptr(snap.get("ant2")),
                    gains=_ptr(snap.get("gains")), n_row=int(snap["uvw"].shape[0]))


def host_snapshot_struct(snap: dict) -> Snapshot:
    """Descriptor of a snapshot whose arrays are torch tensors in host memory
    (page-locked for asynchronous copies: ``pin_memory()``)."""
    import torch
    kinds = {"uvw": torch.float64, "vis": torch.complex64, "freq": torch.float64, "flag": torch.uint8,
             "weight": torch.float32, "ant1": torch.int32, "ant2": torch.int32, "gains": torch.complex64}
    for k, dt in kinds.items():
        t = snap.get(k)
        if t is None:
            if k in ("uvw", "vis", "freq") and snap["uvw"].shape[0] > 0:
                raise ValueError(f"snapshot is missing {k}")
            continue
        if not isinstance(t, torch.Tensor) or t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise TypeError(f"snapshot[{k!r}] must be a contiguous {dt} host tensor")
    return Snapshot(uvw=_ptr(snap["uvw"]), vis=_ptr(snap["vis"]), flag=_ptr(snap.get("flag")),
                    weight=_ptr(snap.get("weight")), freq=_ptr(snap["freq"]),
                    ant1=_ptr(snap.get("ant1")), ant2=_ptr(snap.get("ant2")),
                    gains=_ptr(snap.get("gains")), n_row=int(snap["uvw"].shape[0]))


class Imager:
    """One libtoi context: workspace for N x N images of a given visibility shape."""

    def __init__(self, n_pix: int, cell_deg: float, n_row_max: int, n_chan: int, n_corr: int, *,
                 mode: int = 3, n_slab: int = 0, cheb_k: int = 0, max_planes: int = 0, n_ant: int = 0,
                 tile: int = 32, corr_mask: int = 0, alpha_target: float = 10.0,
                 cheb_gamma: float = 1e-2, bin_cap: int = 0, device=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        L = lib()
        p = Params()
        _check(L.toi_params_default(ctypes.byref(p), n_pix, cell_deg, n_row_max, n_chan, n_corr))
        p.mode, p.n_slab, p.cheb_k, p.max_planes = mode, n_slab, cheb_k, max_planes
        p.n_ant, p.tile, p.corr_mask = n_ant, tile, corr_mask
        p.alpha_target, p.cheb_gamma = alpha_target, cheb_gamma
        p.bin_cap = bin_cap
        self.params = p
        self.n_pix, self.tile = n_pix, tile
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.toi_create(ctypes.byref(p), ctypes.c_void_p(self._stream()), ctypes.byref(h)))
        self.ctx = h
        # bumped by every call that runs sample prep or binning (grid, image_batch,
        # ingest, tune): the per-snapshot state the adjoint reads then belongs to
        # another snapshot
        self._gen = 0
        # held by the instance: at interpreter exit the module's globals may be
        # cleared before a remaining Imager is collected
        self._destroy = L.toi_destroy

    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def _sync_stream(self):
        _check(lib().toi_set_stream(self.ctx, ctypes.c_void_p(self._stream())), self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            self._destroy(self.ctx)
            self.ctx = None

    __del__ = close

    def grid(self, snap: dict):
        self._sync_stream()
        self._snap = snapshot_struct(snap)
        self._gen += 1
        _check(lib().toi_grid(self.ctx, ctypes.byref(self._snap)), self.ctx)

    def image(self, out=None, tplane: bool = False):
        t = self.torch
        N = self.n_pix
        if out is None:
            out = t.empty((N, N), dtype=t.float32, device=self.device)
        tp = t.empty((N, N), dtype=t.float32, device=self.device) if tplane else None
        self._sync_stream()
        _check(lib().toi_image(self.ctx, _ptr(out), _ptr(tp)), self.ctx)
        return (out, tp) if tplane else out

    def degrid(self, grad_image, snap: dict, want_vis=True, want_gains=False):
        t = self.torch
        s = snapshot_struct(snap)
        gv = t.empty_like(snap["vis"]) if want_vis else None
        gg = t.empty_like(snap["gains"]) if want_gains else None
        self._sync_stream()
        _check(lib().toi_degrid(self.ctx, _ptr(grad_image.contiguous()), ctypes.byref(s), _ptr(gv),
                                _ptr(gg)), self.ctx)
        return gv, gg

    def tlisi(self, a, b, c, out=None):
        t = self.torch
        T = self.n_pix // self.tile
        if out is None:
            out = t.empty((T, T), dtype=t.float32, device=self.device)
        self._sync_stream()
        _check(lib().fitrig_tlisi(self.ctx, _ptr(a), _ptr(b), _ptr(c), _ptr(out)), self.ctx)
        return out

    def detect(self, window, t_index: int, max_boxes: int = 256):
        t = self.torch
        boxes = t.zeros((max_boxes, 5), dtype=t.int32, device=self.device)
        n = t.zeros((1,), dtype=t.int32, device=self.device)
        self._sync_stream()
        _check(lib().fitrig_detect(self.ctx, _ptr(window.contiguous()), t_index, _ptr(boxes), max_boxes,
                                   _ptr(n)), self.ctx)
        return boxes, n

    def detect_cube(self, cube, t_index: int, max_boxes: int = 256):
        """Whole-run detection over a (n_maps, T, T) tLISI cube on the device."""
        t = self.torch
        boxes = t.zeros((max_boxes, 5), dtype=t.int32, device=self.device)
        n = t.zeros((1,), dtype=t.int32, device=self.device)
        c = cube.contiguous()
        self._sync_stream()
        _check(lib().fitrig_detect_cube(self.ctx, _ptr(c), int(c.shape[0]), t_index, _ptr(boxes), max_boxes,
                                        _ptr(n)), self.ctx)
        return boxes, n

    def localise(self, img_a, img_b, boxes, ra0_deg: float, dec0_deg: float, morph: bool = True):
        """Positions of the candidates in ``boxes`` (device i32 [n, 5]) in img_b - img_a:
        a device f64 [n, 8] tensor (valid, j1, j2, ra, dec, peak, sigma, pixels)."""
        t = self.torch
        bx = boxes.to(t.int32).contiguous()
        out = t.zeros((bx.shape[0], 8), dtype=t.float64, device=self.device)
        self._sync_stream()
        _check(lib().fitrig_localise(self.ctx, _ptr(img_a.contiguous()), _ptr(img_b.contiguous()), _ptr(bx),
                                     int(bx.shape[0]), float(ra0_deg), float(dec0_deg), 1 if morph else 0,
                                     _ptr(out)), self.ctx)
        return out

    def strongest_map(self, cube, boxes):
        """Per box, the index of the tLISI map with the smallest sum over its tiles."""
        t = self.torch
        bx = boxes.to(t.int32).contiguous()
        k = t.zeros((bx.shape[0],), dtype=t.int32, device=self.device)
        c = cube.contiguous()
        self._sync_stream()
        _check(lib().fitrig_strongest_map(self.ctx, _ptr(c), int(c.shape[0]), _ptr(bx), int(bx.shape[0]),
                                          _ptr(k)), self.ctx)
        return k

    def image_batch(self, snaps, images_out, tlisi_out=None):
        arr = (Snapshot * len(snaps))(*[snapshot_struct(s) for s in snaps])
        self._keep = arr
        self._sync_stream()
        self._gen += 1
        _check(lib().toi_image_batch(self.ctx, arr, len(snaps), _ptr(images_out), _ptr(tlisi_out)),
               self.ctx)

    def batch_inputs(self, n: int, flags=False, weights=False, gains=False):
        """Reserve n context-owned input slots (toi_batch_inputs); returns their
        descriptors (kept by the Imager for image_batch_slots)."""
        arrays = (INPUT_FLAG if flags else 0) | (INPUT_WEIGHT if weights else 0) | (INPUT_GAINS if gains else 0)
        arr = (Snapshot * n)()
        _check(lib().toi_batch_inputs(self.ctx, n, arrays, arr), self.ctx)
        self._slots = arr
        return arr

    def batch_fill(self, slot: int, snap: dict):
        """Copy a device snapshot into input slot `slot` on torch's current stream."""
        s = snapshot_struct(snap)
        self._sync_stream()
        _check(lib().toi_batch_fill(self.ctx, slot, ctypes.byref(s)), self.ctx)

    def image_batch_slots(self, n: int, images_out, tlisi_out=None):
        """toi_image_batch on the first n input slots (the same descriptors each call)."""
        self._sync_stream()
        self._gen += 1
        _check(lib().toi_image_batch(self.ctx, self._slots, n, _ptr(images_out), _ptr(tlisi_out)), self.ctx)

    def batch_info(self):
        """(graphs captured, graphs launched) by toi_image_batch on this context."""
        cap, lau = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().toi_batch_info(self.ctx, ctypes.byref(cap), ctypes.byref(lau)), self.ctx)
        return cap.value, lau.value

    def ingest(self, host_snaps, images_out, tlisi_out=None):
        """Image snapshots held in host memory, copies overlapped with the imaging."""
        arr = (Snapshot * len(host_snaps))(*[host_snapshot_struct(s) for s in host_snaps])
        self._keep_ingest = (arr, host_snaps)
        self._sync_stream()
        self._gen += 1
        _check(lib().toi_ingest(self.ctx, arr, len(host_snaps), _ptr(images_out), _ptr(tlisi_out)), self.ctx)

    def profile(self, enable: bool = True, stages=None):
        """Start (clearing the totals) or stop per-stage HIP-event timing: every
        stage, or only the named ones (names as in ``STAGES``)."""
        mask = 0
        if enable:
            mask = (1 << len(STAGES)) - 1 if stages is None else sum(1 << STAGES.index(n) for n in stages)
        _check(lib().toi_profile_enable(self.ctx, mask), self.ctx)

    def profile_read(self) -> dict:
        """Synchronise; {stage: (total ms, launches)} of the timed stages."""
        ms = (ctypes.c_double * len(STAGES))()
        n = (ctypes.c_int32 * len(STAGES))()
        self._sync_stream()
        _check(lib().toi_profile_read(self.ctx, ms, n), self.ctx)
        return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}

    def tune(self, snap: dict):
        """Time every gridder variant on ``snap``, keep the fastest; (variant, [ms per variant])."""
        desc = snapshot_struct(snap)
        v = ctypes.c_int32()
        ms = (ctypes.c_float * TUNE_VARIANTS)()
        self._sync_stream()
        self._gen += 1
        _check(lib().toi_tune(self.ctx, ctypes.byref(desc), ctypes.byref(v), ms), self.ctx)
        return v.value, list(ms)

    def set_tuning(self, variant: int):
        _check(lib().toi_set_tuning(self.ctx, variant), self.ctx)

    def bin_info(self) -> dict:
        """Synchronise; the last gridded snapshot's bin-list entries, occupied
        (plane group, tile) pairs, occupied (plane group, tile row) pairs and work units."""
        v = [ctypes.c_int64() for _ in range(4)]
        self._sync_stream()
        _check(lib().toi_bin_info(self.ctx, *[ctypes.byref(x) for x in v]), self.ctx)
        return dict(zip(("entries", "tiles", "tile_rows", "units"), (x.value for x in v)))

    def plan_info(self) -> dict:
        V = (ctypes.c_double * 9)()
        om, ws = ctypes.c_double(), ctypes.c_double()
        ns, k = ctypes.c_int32(), ctypes.c_int32()
        st = ctypes.c_uint32()
        self._sync_stream()
        _check(lib().toi_plan_info(self.ctx, V, ctypes.byref(om), ctypes.byref(ws), ctypes.byref(ns),
                                   ctypes.byref(k), ctypes.byref(st)), self.ctx)
        import numpy as np
        return dict(V=np.array(V[:]).reshape(3, 3), omega=om.value, wsum=ws.value, n_slab=ns.value,
                    K=k.value, status=st.value)


def tlisi_noalloc(a, b, c, tile: int, out):
    """fitrig_tlisi_noalloc: the tLISI map of three device images into the
    caller's ``out`` (float32 [N/tile][N/tile]) on torch's current stream, with
    no context and no allocation (the library's static per-device scratch)."""
    import torch
    n_pix = int(a.shape[-1])
    stream = torch.cuda.current_stream(a.device).cuda_stream
    _check(lib().fitrig_tlisi_noalloc(_ptr(a), _ptr(b), _ptr(c), n_pix, int(tile), _ptr(out),
                                      ctypes.c_void_p(stream)))
    return out


def to_device(snap: dict, device="cuda") -> dict:
    """Copy a host snapshot (numpy arrays, as produced by synth_inputs) to GPU tensors."""
    import numpy as np
    import torch
    out = {}
    for k in ("uvw", "vis", "flag", "weight", "freq", "ant1", "ant2", "gains"):
        v = snap.get(k)
        out[k] = None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to(device)
    return out


def to_host(snap: dict, pinned: bool = True) -> dict:
    """A host snapshot (numpy arrays) as torch host tensors for ``Imager.ingest``,
    page-locked unless ``pinned`` is False."""
    import numpy as np
    import torch
    out = {}
    for k in ("uvw", "vis", "flag", "weight", "freq", "ant1", "ant2", "gains"):
        v = snap.get(k)
        if v is None:
            out[k] = None
            continue
        t = torch.from_numpy(np.ascontiguousarray(v))
        out[k] = t.pin_memory() if pinned else t.clone()
    return out


def _autograd_function():
    import torch

    class TOIImage(torch.autograd.Function):
        """Differentiable snapshot image: forward = toi_grid + toi_image, backward = toi_degrid.

        Gradients follow PyTorch's convention for complex inputs of a real loss
        (dL/dRe + i dL/dIm) and are returned for ``vis`` and, when given, ``gains``.
        """

        @staticmethod
        def forward(ctx, vis, gains, imager, snap):
            s = dict(snap)
            s["vis"] = vis.contiguous()
            if gains is not None:
                s["gains"] = gains.contiguous()
            imager.grid(s)
            img = imager.image()
            ctx.imager, ctx.snap, ctx.has_gains, ctx.gen = imager, s, gains is not None, imager._gen
            return img

        @staticmethod
        def backward(ctx, grad_img):
            im, s = ctx.imager, ctx.snap
            if im._gen != ctx.gen:
                im.grid(s)             # the context prepared another snapshot since: re-establish this one's
                ctx.gen = im._gen      # plan, records and bins
            want_g = ctx.has_gains and ctx.needs_input_grad[1]
            gv, gg = im.degrid(grad_img.contiguous(), s, want_vis=ctx.needs_input_grad[0], want_gains=want_g)
            return gv, gg, None, None

    return TOIImage


_TOIImage = None


def toi_image(imager: "Imager", snap: dict, vis=None, gains=None):
    """Image one snapshot with autograd support for ``vis`` (and ``gains``)."""
    global _TOIImage
    if _TOIImage is None:
        _TOIImage = _autograd_function()
    return _TOIImage.apply(snap["vis"] if vis is None else vis, gains if gains is not None else snap.get("gains"),
                           imager, snap)
