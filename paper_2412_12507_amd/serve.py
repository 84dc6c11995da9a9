"""Python client of the continuous-batching server (gut_serve_* in gut.h).

The server keeps a scene resident, admits multi-camera requests by memory,
merges queued requests into batches and renders each batch with one
persistent launch per shutter type on one of its slot streams.  This module
only marshals arguments and keeps the Python objects (scene tensors, output
images) alive while the server uses them.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L
from .raster import GaussianScene


class Server:
    def __init__(self, scene: GaussianScene, params: dict | None = None,
                 mem_budget_bytes: int = 16 << 30, max_slots: int = 4, max_batch_cams: int = 8):
        self._lib = L.load()
        self.scene = scene                      # borrowed by the server: keep alive
        self._ss = scene.struct()
        self._ps = L.params_struct(params)
        self._h = C.c_void_p()
        L.check(self._lib.gut_serve_create(L.ref(self._ss), L.ref(self._ps), int(mem_budget_bytes),
                                           int(max_slots), int(max_batch_cams), C.byref(self._h)),
                "gut_serve_create")
        self._outs: dict[int, list] = {}

    def submit(self, cams, outs=None):
        """Enqueue one request; returns (request id, list of [H,W,3] output tensors)."""
        if outs is None:
            outs = [torch.empty(int(c["height"]), int(c["width"]), 3, device=self.scene.means.device)
                    for c in cams]
        arr = L.camera_array(cams)
        ptrs = (C.c_void_p * len(cams))(*[o.data_ptr() for o in outs])
        rid = C.c_uint64(0)
        L.check(self._lib.gut_serve_submit(self._h, arr, len(cams), ptrs, C.byref(rid)),
                "gut_serve_submit")
        self._outs[rid.value] = outs
        return rid.value, outs

    def poll(self, rid: int) -> bool:
        done = C.c_int32(0)
        L.check(self._lib.gut_serve_poll(self._h, C.c_uint64(rid), C.byref(done)), "gut_serve_poll")
        return bool(done.value)

    def wait(self, rid: int):
        L.check(self._lib.gut_serve_wait(self._h, C.c_uint64(rid)), "gut_serve_wait")
        return self._outs.pop(rid, None)

    def latency_ms(self, rid: int) -> float:
        ms = C.c_double(0)
        L.check(self._lib.gut_serve_latency(self._h, C.c_uint64(rid), C.byref(ms)),
                "gut_serve_latency")
        return ms.value

    def stats(self) -> dict:
        m = L.ServeMetrics()
        L.check(self._lib.gut_serve_stats(self._h, L.ref(m)), "gut_serve_stats")
        return {k: getattr(m, k) for k, _ in L.ServeMetrics._fields_}

    def reset_stats(self):
        L.check(self._lib.gut_serve_reset_stats(self._h), "gut_serve_reset_stats")

    def close(self):
        if self._h:
            L.check(self._lib.gut_serve_destroy(self._h), "gut_serve_destroy")
            self._h = C.c_void_p()
            self._outs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def render_sequential(scene: GaussianScene, cams, params=None):
    """The one-request-at-a-time reference: each camera rendered alone through
    gut_project -> gut_bin -> gut_render, synchronously."""
    from . import raster as R
    out = []
    for cam in cams:
        _, _, img = R.forward(scene, [cam], params)
        out.append(img.images("rgb")[0])
    torch.cuda.synchronize()
    return out
