"""Python front end of the gmmsp library: PyTorch supplies device memory and
the stream, libgmmsp.so does every step of the method."""
from __future__ import annotations

import ctypes
from ctypes import byref, c_double, c_int32, c_int64, c_size_t, c_void_p
from typing import Sequence

import numpy as np
import torch

from . import _lib
from ._lib import GmmspGridInfo, GmmspParams, check, lib


def make_params(W: int, H: int, K: int = 0, vx: int = 0, vy: int = 0, eps_s: float = 2.0,
                eps_c: float = 8.0, lam: float = 8.0, cov_mode: int = 0,
                n_min: float = 1e-3) -> GmmspParams:
    return GmmspParams(W, H, K, vx, vy, eps_s, eps_c, lam, cov_mode, n_min)


def grid(W: int, H: int, K: int = 0, vx: int = 0, vy: int = 0) -> GmmspGridInfo:
    """Seed grid by Eqs. vxy and nxyK (host-only library call)."""
    g = GmmspGridInfo()
    check(lib().gmmsp_grid(byref(make_params(W, H, K, vx, vy)), byref(g)))
    return g


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def srgb8_to_lab(rgb: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """8-bit sRGB (..., 3) uint8 on the GPU -> CIELAB (..., 3) float32 (D65)."""
    if rgb.dtype != torch.uint8 or not rgb.is_contiguous() or rgb.shape[-1] != 3 or not rgb.is_cuda:
        raise ValueError("rgb must be a contiguous (..., 3) uint8 tensor on the GPU")
    if out is None:
        out = torch.empty(rgb.shape, dtype=torch.float32, device=rgb.device)
    s = torch.cuda.current_stream(rgb.device).cuda_stream
    check(lib().gmmsp_srgb8_to_lab(c_void_p(_ptr(rgb)), rgb.numel() // 3, c_void_p(_ptr(out)),
                                   c_void_p(s)))
    return out


class GMMSP:
    """A batch of images (one image is a batch of one) bound to a workspace.

    ``sizes``: sequence of (W, H); ``K`` (or ``v``, an int or a (vx, vy) tuple):
    one value for all images, or a list with one value per image.  ``cov_mode``:
    0 split colour blocks, 1 the 3x3 colour block, 2 the full 5x5 covariance,
    3 grayscale images.  Inputs are packed float32 tensors on the device, three
    channels (L, a, b) per pixel, one (the intensity) with cov_mode 3; image b
    starts at pixel offset ``pix_off[b]``."""

    def __init__(self, sizes: Sequence[tuple], K=None, v=None, eps_s: float = 2.0,
                 eps_c: float = 8.0, lam: float = 8.0, n_min: float = 1e-3,
                 device="cuda", cov_mode: int = 0):
        n = len(sizes)
        # a list gives one value per image; a (vx, vy) tuple is one spacing for all
        Ks = K if isinstance(K, list) else [K] * n
        vs = v if isinstance(v, list) else [v] * n
        arr = (GmmspParams * n)()
        for b, (W, H) in enumerate(sizes):
            vb = vs[b]
            vx, vy = (vb if isinstance(vb, (list, tuple)) else (vb, vb)) if vb else (0, 0)
            arr[b] = make_params(W, H, Ks[b] or 0, vx, vy, eps_s, eps_c, lam, cov_mode, n_min)
        if cov_mode not in _lib.THETA_ROWS:
            raise ValueError("cov_mode must be 0, 1, 2 or 3")
        self.params = arr
        self.cov_mode = cov_mode
        self.theta_row = _lib.THETA_ROWS[cov_mode]
        self.channels = 1 if cov_mode == 3 else 3   # grayscale: one float per pixel
        self.n_images = n
        self.device = torch.device(device)
        nbytes = c_size_t(0)
        check(lib().gmmsp_workspace_bytes(n, arr, byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        h = c_void_p()
        check(lib().gmmsp_create(n, arr, c_void_p(_ptr(self.workspace)), nbytes.value,
                                 c_void_p(self._stream()), byref(h)))
        self.handle = h
        ni, npx, nsp = c_int32(), c_int64(), c_int64()
        check(lib().gmmsp_batch_info(h, byref(ni), byref(npx), byref(nsp)))
        self.n_pixels = npx.value
        self.n_superpixels = nsp.value
        self.grids = []
        for b in range(n):
            g = GmmspGridInfo()
            check(lib().gmmsp_image_grid(h, b, byref(g)))
            self.grids.append(g)
        self.sizes = [tuple(s) for s in sizes]
        self.pix_off = np.concatenate([[0], np.cumsum([W * H for W, H in sizes])]).astype(np.int64)
        self.sp_off = np.concatenate([[0], np.cumsum([g.K for g in self.grids])]).astype(np.int64)

    # -- plumbing ------------------------------------------------------------
    def _stream(self) -> int:
        return torch.cuda.current_stream(self.device).cuda_stream

    def _lab(self, lab: torch.Tensor, channels: int | None = None) -> c_void_p:
        ch = self.channels if channels is None else channels
        if lab.dtype != torch.float32 or not lab.is_contiguous() or lab.device != self.device:
            raise ValueError("lab must be a contiguous float32 tensor on the handle's device")
        if lab.numel() != ch * self.n_pixels:
            raise ValueError(f"lab has {lab.numel()} floats, expected {ch * self.n_pixels}")
        return c_void_p(_ptr(lab))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().gmmsp_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the method ------------------------------------------------------------
    def init_seeds(self, lab: torch.Tensor):
        check(lib().gmmsp_init_seeds(self.handle, self._lab(lab), c_void_p(self._stream())))

    def set_params(self, rows) -> None:
        """theta rows (n_superpixels, 13): numpy (host) or a float64 device tensor."""
        if isinstance(rows, torch.Tensor) and rows.device.type == "cuda":
            if rows.dtype != torch.float64 or not rows.is_contiguous() or \
                    rows.shape != (self.n_superpixels, self.theta_row):
                raise ValueError(f"theta must be a contiguous (n_sp, {self.theta_row}) float64 tensor")
            check(lib().gmmsp_set_params_dev(self.handle, c_void_p(_ptr(rows)),
                                             c_void_p(self._stream())))
            return
        a = np.ascontiguousarray(np.asarray(rows, dtype=np.float64))
        if a.shape != (self.n_superpixels, self.theta_row):
            raise ValueError(f"theta must have shape (n_superpixels, {self.theta_row})")
        check(lib().gmmsp_set_params(self.handle, c_void_p(a.ctypes.data),
                                     c_void_p(self._stream())))

    def get_params(self) -> np.ndarray:
        out = np.empty((self.n_superpixels, self.theta_row), dtype=np.float64)
        check(lib().gmmsp_get_params(self.handle, c_void_p(out.ctypes.data),
                                     c_void_p(self._stream())))
        return out

    def em_iterate(self, lab: torch.Tensor, max_iters: int, rel_tol: float = 0.0) -> np.ndarray:
        it = np.zeros(self.n_images, dtype=np.int32)
        check(lib().gmmsp_em_iterate(self.handle, self._lab(lab), int(max_iters),
                                     float(rel_tol), c_void_p(it.ctypes.data),
                                     c_void_p(self._stream())))
        return it

    def ll_history(self, b: int = 0) -> np.ndarray:
        out = np.empty(_lib.LL_CAP, dtype=np.float64)
        n = c_int32()
        check(lib().gmmsp_ll_history(self.handle, b, c_void_p(out.ctypes.data), _lib.LL_CAP,
                                     byref(n), c_void_p(self._stream())))
        return out[:n.value].copy()

    def label(self, lab: torch.Tensor, labels: torch.Tensor | None = None, want_ll=True):
        if labels is None:
            labels = torch.empty(self.n_pixels, dtype=torch.int32, device=self.device)
        ll = np.zeros(self.n_images, dtype=np.float64)
        check(lib().gmmsp_label(self.handle, self._lab(lab), c_void_p(_ptr(labels)),
                                c_void_p(ll.ctypes.data) if want_ll else None,
                                c_void_p(self._stream())))
        return labels, ll

    def export_responsibilities(self, lab: torch.Tensor) -> torch.Tensor:
        R = torch.zeros((self.n_pixels, 9), dtype=torch.float32, device=self.device)
        check(lib().gmmsp_export_responsibilities(self.handle, self._lab(lab),
                                                  c_void_p(_ptr(R)), c_void_p(self._stream())))
        return R

    def export_candidates(self) -> torch.Tensor:
        c = torch.full((self.n_pixels, 9), -3, dtype=torch.int32, device=self.device)
        check(lib().gmmsp_export_candidates(self.handle, c_void_p(_ptr(c)),
                                            c_void_p(self._stream())))
        return c

    # -- schedules, autotuning and graph replay --------------------------------
    def set_schedule(self, waves_per_cell: int):
        check(lib().gmmsp_set_schedule(self.handle, int(waves_per_cell)))

    def get_schedule(self) -> int:
        w = c_int32()
        check(lib().gmmsp_get_schedule(self.handle, byref(w)))
        return w.value

    def set_estep_kernel(self, kind: int):
        """0: one pixel per lane; 1: one candidate slot per lane (cov_mode 0)."""
        check(lib().gmmsp_set_estep_kernel(self.handle, int(kind)))

    def get_estep_kernel(self) -> int:
        k = c_int32()
        check(lib().gmmsp_get_estep_kernel(self.handle, byref(k)))
        return k.value

    def set_slot_rows(self, rows: int):
        """Rows per chunk (tile height) of the slot-lane pass."""
        check(lib().gmmsp_set_slot_rows(self.handle, int(rows)))

    def get_slot_rows(self) -> int:
        r = c_int32()
        check(lib().gmmsp_get_slot_rows(self.handle, byref(r)))
        return r.value

    def schedule(self) -> dict:
        """The schedule in effect: statistics-pass kind, rows per chunk, waves
        per cell, gather lanes, and whether T-mode passes run as one
        persistent launch."""
        return {"estep_kernel": self.get_estep_kernel(), "rows_per_chunk": self.get_slot_rows(),
                "waves_per_cell": self.get_schedule(), "gather_lanes": self.get_gather_lanes(),
                "persistent": self.get_persistent()}

    def set_gather_lanes(self, lanes_per_superpixel: int):
        check(lib().gmmsp_set_gather_lanes(self.handle, int(lanes_per_superpixel)))

    def get_gather_lanes(self) -> int:
        n = c_int32()
        check(lib().gmmsp_get_gather_lanes(self.handle, byref(n)))
        return n.value

    def set_graph_passes(self, passes: int):
        check(lib().gmmsp_set_graph_passes(self.handle, int(passes)))

    def set_persistent(self, on: bool):
        """T-mode passes (no stop rule) of the slot-lane pass as one persistent
        cooperative launch per em_iterate call."""
        check(lib().gmmsp_set_persistent(self.handle, 1 if on else 0))

    def get_persistent(self) -> int:
        v = c_int32()
        check(lib().gmmsp_get_persistent(self.handle, byref(v)))
        return v.value

    def geometry_key(self) -> str:
        dev = torch.cuda.get_device_name(self.device)
        grids = ";".join(f"{W}x{H}/{g.vx}x{g.vy}" for (W, H), g in zip(self.sizes, self.grids))
        import hashlib
        return (f"{dev}|{self.n_images}|m{self.cov_mode}|" +
                hashlib.sha256(grids.encode()).hexdigest()[:16])

    def autotune(self, lab: torch.Tensor, passes: int = 3, cache: str | None = "default") -> int:
        """Pick the statistics-pass schedule (kind, rows per chunk, waves per
        cell), then the lanes per superpixel of the gather, then per-pass or
        persistent T-mode launches, by timing them on this batch (native
        loops in the library); results are cached by batch
        geometry in a JSON file (~/.cache/gmmsp/schedules.json unless another
        path or None is given).  Returns the waves per cell.  Leaves the handle
        initialised by init_seeds."""
        import json
        import os
        path = None
        if cache == "default":
            path = os.path.join(os.path.expanduser("~"), ".cache", "gmmsp", "schedules.json")
        elif cache:
            path = cache
        key = self.geometry_key()
        table = {}
        if path and os.path.exists(path):
            try:
                with open(path) as f:
                    table = json.load(f)
            except (OSError, ValueError):
                table = {}
        entry = table.get(key)
        if entry and "estep_kernel" in entry:
            self.set_estep_kernel(int(entry["estep_kernel"]))
            if int(entry.get("rows_per_chunk", 0)):
                self.set_slot_rows(int(entry["rows_per_chunk"]))
            self.set_schedule(int(entry["waves_per_cell"]))
            self.set_gather_lanes(int(entry.get("lanes_per_superpixel", 1)))
            self.set_persistent(bool(entry.get("persistent", 0)))
            self.init_seeds(lab)
            self.tune_cached = True
            return self.get_schedule()
        self.tune_cached = False
        ms = np.zeros(_lib.TUNE_CANDIDATES)
        w = c_int32()
        check(lib().gmmsp_autotune(self.handle, self._lab(lab), int(passes),
                                   c_void_p(ms.ctypes.data), byref(w), c_void_p(self._stream())))
        # candidate 3 v + w: v = 0..2 slot-lane rows values (largest first), 3 pixel-lane
        self.tune_ms = {f"v{v}w{(1, 2, 4)[i]}": float(ms[3 * v + i])
                        for v in range(4) for i in range(3) if ms[3 * v + i] >= 0}
        gms = np.zeros(3)
        lanes = c_int32()
        check(lib().gmmsp_autotune_gather(self.handle, self._lab(lab), int(passes),
                                          c_void_p(gms.ctypes.data), byref(lanes),
                                          c_void_p(self._stream())))
        self.tune_gather_ms = dict(zip((1, 4, 16), gms.tolist()))
        pms = np.zeros(4)
        pers = c_int32()
        # the launch form's fixed cost is amortised over the T passes of a run:
        # time at least the paper's T = 10
        check(lib().gmmsp_autotune_persistent(self.handle, self._lab(lab), max(int(passes), 10),
                                              c_void_p(pms.ctypes.data), byref(pers),
                                              c_void_p(self._stream())))
        # per-pass launches, then the persistent launch per rows value (largest first)
        self.tune_persistent_ms = {k: float(v) for k, v in
                                   zip(("per_pass", "r0", "r1", "r2"), pms) if v >= 0}
        if path:
            table[key] = {"estep_kernel": self.get_estep_kernel(),
                          "rows_per_chunk": self.get_slot_rows(),
                          "waves_per_cell": w.value, "ms": self.tune_ms,
                          "lanes_per_superpixel": lanes.value, "gather_ms": self.tune_gather_ms,
                          "persistent": pers.value, "persistent_ms": self.tune_persistent_ms}
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(table, f, indent=1)
        return w.value

    def profile(self, enable: bool = True):
        check(lib().gmmsp_profile_enable(self.handle, 1 if enable else 0))

    def profile_read(self, reset: bool = True) -> dict:
        ms, n, px, pr = c_double(), c_int32(), c_int64(), c_int64()
        check(lib().gmmsp_profile_read(self.handle, byref(ms), byref(n), byref(px), byref(pr),
                                       1 if reset else 0))
        return dict(estep_ms=ms.value, launches=n.value, pixel_evals=px.value,
                    pair_evals=pr.value)

    # -- learned warm start ----------------------------------------------------
    def ws_attach(self):
        """Allocate (torch) and attach the warm-start workspace."""
        if getattr(self, "ws_workspace", None) is not None:
            return
        nbytes = c_size_t(0)
        check(lib().gmmsp_ws_workspace_bytes(self.handle, byref(nbytes)))
        self.ws_workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        check(lib().gmmsp_ws_attach(self.handle, c_void_p(_ptr(self.ws_workspace)), nbytes.value,
                                    c_void_p(self._stream())))

    def _params(self, params: torch.Tensor) -> c_void_p:
        if params.dtype != torch.float32 or not params.is_contiguous() or \
                params.numel() != _lib.WS_NPARAM or params.device != self.device:
            raise ValueError(f"parameters must be {_lib.WS_NPARAM} contiguous float32 on the device")
        return c_void_p(_ptr(params))

    def ws_features(self, lab: torch.Tensor):
        check(lib().gmmsp_ws_features(self.handle, self._lab(lab), c_void_p(self._stream())))

    def ws_forward(self, params: torch.Tensor, b0: int = 0, b1: int | None = None):
        b1 = self.n_images if b1 is None else b1
        check(lib().gmmsp_ws_forward(self.handle, self._params(params), b0, b1,
                                     c_void_p(self._stream())))

    def ws_apply(self, lab: torch.Tensor, mask: int = _lib.WS_ALL_OUTPUTS):
        check(lib().gmmsp_ws_apply(self.handle, self._lab(lab), int(mask),
                                   c_void_p(self._stream())))

    def ws_apply_guarded(self, lab: torch.Tensor, mask: int = _lib.WS_ALL_OUTPUTS,
                         want_flags: bool = False):
        """ws_apply, keeping the grid seeds for every image whose L(theta^0)
        under the network is lower (or not finite).  With want_flags, returns
        the per-image fallback flags (synchronises)."""
        flags = np.zeros(self.n_images, dtype=np.int32) if want_flags else None
        check(lib().gmmsp_ws_apply_guarded(self.handle, self._lab(lab), int(mask),
                                           c_void_p(flags.ctypes.data) if want_flags else None,
                                           c_void_p(self._stream())))
        return flags

    def ws_targets(self, lab: torch.Tensor):
        check(lib().gmmsp_ws_targets(self.handle, self._lab(lab), c_void_p(self._stream())))

    def ws_train_step(self, params, m, v, step: int, lr: float, b0: int = 0, b1=None,
                      want_loss: bool = True):
        b1 = self.n_images if b1 is None else b1
        loss = c_double(0.0)
        for t in (m, v):
            self._params(t)
        check(lib().gmmsp_ws_train_step(self.handle, self._params(params), c_void_p(_ptr(m)),
                                        c_void_p(_ptr(v)), int(step), float(lr), b0, b1,
                                        byref(loss) if want_loss else None,
                                        c_void_p(self._stream())))
        return loss.value if want_loss else None

    def ws_read(self, name: str) -> np.ndarray:
        idx, dt, ch = _lib.WS_BUFFERS[name]
        n = _lib.WS_NPARAM if ch is None else self.n_superpixels * ch
        if dt == "bf16":
            raw = np.empty(n, dtype=np.uint16)
            check(lib().gmmsp_ws_read(self.handle, idx, c_void_p(raw.ctypes.data), raw.nbytes,
                                      c_void_p(self._stream())))
            out = (raw.astype(np.uint32) << 16).view(np.float32)
        else:
            out = np.empty(n, dtype=np.float32)
            check(lib().gmmsp_ws_read(self.handle, idx, c_void_p(out.ctypes.data), out.nbytes,
                                      c_void_p(self._stream())))
        return out if ch is None else out.reshape(self.n_superpixels, ch)

    def ws_write(self, name: str, values: np.ndarray):
        idx, dt, ch = _lib.WS_BUFFERS[name]
        if dt != "float32":
            raise ValueError("only float32 buffers can be written")
        a = np.ascontiguousarray(np.asarray(values, dtype=np.float32))
        check(lib().gmmsp_ws_write(self.handle, idx, c_void_p(a.ctypes.data), a.nbytes,
                                   c_void_p(self._stream())))

    # -- connectivity post-processing (Algorithm 1, last step) ----------------
    def connectivity(self, lab: torch.Tensor, labels: torch.Tensor,
                     out: torch.Tensor | None = None, compact: bool = False):
        """Merge the small disconnected segments of `labels` (int32 per pixel of
        the batch) into colour-nearest neighbours.  Returns (out, counts): out
        holds, per pixel, the image-local raster index of its final segment's
        first pixel (or, with compact, the segment's rank 0 .. final - 1 in its
        image); counts (n_images, 4): segments, small, merged, final."""
        if labels.dtype != torch.int32 or not labels.is_contiguous() or \
                labels.numel() != self.n_pixels or labels.device != self.device:
            raise ValueError("labels must be a contiguous int32 tensor of n_pixels on the handle's device")
        if out is None:
            out = torch.empty_like(labels)
        nbytes = c_size_t(0)
        check(lib().gmmsp_conn_workspace_bytes(self.handle, byref(nbytes)))
        ws = getattr(self, "conn_workspace", None)
        if ws is None or ws.numel() < nbytes.value:
            ws = self.conn_workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        counts = np.zeros((self.n_images, 4), dtype=np.int32)
        check(lib().gmmsp_connectivity(self.handle, self._lab(lab, 3), c_void_p(_ptr(labels)),
                                       c_void_p(_ptr(out)), c_void_p(_ptr(ws)), nbytes.value,
                                       1 if compact else 0, c_void_p(counts.ctypes.data),
                                       c_void_p(self._stream())))
        return out, counts

    def conn_workspace_bytes(self) -> int:
        nbytes = c_size_t(0)
        check(lib().gmmsp_conn_workspace_bytes(self.handle, byref(nbytes)))
        return nbytes.value

    def connectivity_static(self, lab: torch.Tensor, labels: torch.Tensor,
                            out: torch.Tensor | None = None, compact: bool = False):
        """connectivity() on the library's own scratch array instead of a
        workspace: the entry point for callers that cannot allocate (one array
        per GPU, at most _lib.CONN_STATIC_BYTES of workspace; calls that
        overlap on one GPU race)."""
        if labels.dtype != torch.int32 or not labels.is_contiguous() or \
                labels.numel() != self.n_pixels or labels.device != self.device:
            raise ValueError("labels must be a contiguous int32 tensor of n_pixels on the handle's device")
        if out is None:
            out = torch.empty_like(labels)
        counts = np.zeros((self.n_images, 4), dtype=np.int32)
        check(lib().gmmsp_connectivity_static(self.handle, self._lab(lab, 3), c_void_p(_ptr(labels)),
                                              c_void_p(_ptr(out)), 1 if compact else 0,
                                              c_void_p(counts.ctypes.data),
                                              c_void_p(self._stream())))
        return out, counts

    # -- accuracy measures (Sec. IV: BR, Eq. ue, Eq. asa) ----------------------
    def metrics(self, labels: torch.Tensor, gt: torch.Tensor, n_gt, n_sp=None):
        """BR, UE, ASA per image of `labels` (int32, values in [0, n_sp[b]),
        by default [0, K_b)) against `gt` (int32, values in [0, n_gt[b])).
        Returns (values (n_images, 3), integer sums (n_images, 4))."""
        for t, name in ((labels, "labels"), (gt, "gt")):
            if t.dtype != torch.int32 or not t.is_contiguous() or t.numel() != self.n_pixels \
                    or t.device != self.device:
                raise ValueError(f"{name} must be a contiguous int32 tensor of n_pixels on the handle's device")
        ngt = np.ascontiguousarray(np.broadcast_to(np.asarray(n_gt, dtype=np.int32), (self.n_images,)))
        nsp = None if n_sp is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(n_sp, dtype=np.int32), (self.n_images,)))
        nsp_p = c_void_p(nsp.ctypes.data) if nsp is not None else None
        nbytes = c_size_t(0)
        check(lib().gmmsp_metrics_workspace_bytes(self.handle, nsp_p, c_void_p(ngt.ctypes.data),
                                                  byref(nbytes)))
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        out = np.zeros((self.n_images, 3), dtype=np.float64)
        sums = np.zeros((self.n_images, 4), dtype=np.int64)
        check(lib().gmmsp_metrics(self.handle, c_void_p(_ptr(labels)), c_void_p(_ptr(gt)), nsp_p,
                                  c_void_p(ngt.ctypes.data), c_void_p(_ptr(ws)), nbytes.value,
                                  c_void_p(out.ctypes.data), c_void_p(sums.ctypes.data),
                                  c_void_p(self._stream())))
        return out, sums

    # -- helpers -------------------------------------------------------------
    def image_slice(self, b: int) -> slice:
        return slice(int(self.pix_off[b]), int(self.pix_off[b + 1]))

    def sp_slice(self, b: int) -> slice:
        return slice(int(self.sp_off[b]), int(self.sp_off[b + 1]))
