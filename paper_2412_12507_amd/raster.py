"""PyTorch-facing API of the 3DGUT rasterizer (argument marshalling only).

  project(scene, cams)            -> Projection  (gut_project)
  bin_tiles(proj, cams)           -> Bins        (gut_bin, grows its pair buffer on demand)
  render(proj, bins, cams)        -> Image       (gut_render)
  render_backward(...)            -> gradients   (gut_render_bwd)
  GutRender / render_gaussians    torch.autograd.Function over the four calls

Tensors live on the current CUDA (HIP) device and every call is issued on
torch's current stream.  Parameters passed here are ACTIVATED (scales > 0,
opacities in (0,1)); wrap raw parameters with exp / sigmoid in torch.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import torch

from . import _lib as L


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class GaussianScene:
    """Activated particle parameters on the GPU (float32, contiguous)."""
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    opacities: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @classmethod
    def from_host(cls, scene, device="cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)
        return cls(f(scene.means), f(scene.scales), f(scene.quats), f(scene.opacities).reshape(-1),
                   f(scene.sh), int(scene.sh_degree))

    def struct(self) -> L.Scene:
        s = L.Scene()
        s.n, s.sh_degree, s.reserved = self.n, self.sh_degree, 0
        s.means, s.scales, s.quats = (t.data_ptr() for t in (self.means, self.scales, self.quats))
        s.opacities, s.sh = self.opacities.data_ptr(), self.sh.data_ptr()
        return s


@dataclass
class Projection:
    rect: torch.Tensor     # [C*n,4] int16
    tiles: torch.Tensor    # [C*n]   int32 (uint32 values)
    depth: torch.Tensor    # [C*n]   float32
    rgb: torch.Tensor      # [C*n,3] float32
    record: torch.Tensor   # [n,16]  float32
    mean2d: torch.Tensor | None = None  # [C*n,2] UT mean (tile culling reads it)
    cov2d: torch.Tensor | None = None   # [C*n,3] UT covariance (debug)
    extent: torch.Tensor | None = None  # [C*n,4] extent ellipse k^2 Sigma' and k (tile culling)
    n: int = 0
    n_cams: int = 1

    def struct(self) -> L.Projected:
        p = L.Projected()
        for k in ("rect", "tiles", "depth", "rgb", "record", "mean2d", "cov2d", "extent"):
            t = getattr(self, k)
            setattr(p, k, None if t is None else t.data_ptr())
        return p


@dataclass
class Bins:
    ranges: torch.Tensor   # [T,2] int32, first 2T entries of the buffer gut_bin writes
    ids: torch.Tensor      # [capacity] int32 (entry ids)
    n_pairs: int
    order: torch.Tensor = None   # [T] int32 render order (the buffer's last T entries)
    workspace: torch.Tensor = field(repr=False, default=None)


@dataclass
class Image:
    rgb: torch.Tensor        # [P_px,3]
    T: torch.Tensor          # [P_px]
    n_contrib: torch.Tensor  # [P_px] int32
    n_eval: torch.Tensor | None
    shapes: list

    def images(self, key="rgb"):
        """Split a concatenated per-pixel output into per-camera [H, W, ...] views."""
        t = getattr(self, key)
        out, o = [], 0
        for (h, w) in self.shapes:
            out.append(t[o:o + h * w].view(h, w, *t.shape[1:]))
            o += h * w
        return out


def num_tiles(cams, params=None) -> int:
    arr = L.camera_array(cams)
    p = L.params_struct(params)
    t = L.load().gut_num_tiles(arr, len(cams), L.ref(p))
    if t < 0:
        raise ValueError("bad cameras")
    return int(t)


def num_pixels(cams) -> int:
    return int(sum(int(c["width"]) * int(c["height"]) for c in cams))


def alloc_projection(n, n_cams, device="cuda", debug=False) -> Projection:
    E = n * n_cams
    mk = lambda *s, dt=torch.float32: torch.empty(*s, dtype=dt, device=device)
    return Projection(rect=mk(E, 4, dt=torch.int16), tiles=mk(E, dt=torch.int32), depth=mk(E),
                      rgb=mk(E, 3), record=mk(max(n, 1), 16),
                      mean2d=mk(E, 2), cov2d=mk(E, 3) if debug else None, extent=mk(E, 4),
                      n=n, n_cams=n_cams)


def project(scene: GaussianScene, cams, params=None, out: Projection | None = None,
            debug=False) -> Projection:
    n, nc = scene.n, len(cams)
    if out is None:
        out = alloc_projection(n, nc, scene.means.device, debug)
    arr = L.camera_array(cams)
    p = L.params_struct(params)
    ss, ps = scene.struct(), out.struct()
    L.check(L.load().gut_project(L.ref(ss), arr, nc, L.ref(p), L.ref(ps), _stream()),
            "gut_project")
    return out


def bin_tiles(proj: Projection, cams, params=None, bins: Bins | None = None,
              capacity: int | None = None) -> Bins:
    """gut_bin; grows the pair buffer and retries if it is too small."""
    lib = L.load()
    n, nc = proj.n, len(cams)
    dev = proj.depth.device
    T = num_tiles(cams, params)
    arr = L.camera_array(cams)
    p = L.params_struct(params)
    if bins is None or bins.ranges.shape[0] != T:
        # [T,2] ranges followed by the [T] render order, in one buffer
        rbuf = torch.empty(3 * T, dtype=torch.int32, device=dev)
        ranges, order = rbuf[:2 * T].view(T, 2), rbuf[2 * T:]
    else:
        ranges, order = bins.ranges, bins.order
    cap = capacity if capacity is not None else (
        bins.ids.shape[0] if bins is not None else max(4096, 16 * n * nc))
    ids = bins.ids if (bins is not None and bins.ids.shape[0] >= cap) else None
    ws = bins.workspace if bins is not None else None
    for _ in range(3):
        if ids is None or ids.shape[0] < cap:
            ids = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        need = lib.gut_bin_workspace_bytes(n, arr, nc, ids.shape[0])
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(int(need), 256), dtype=torch.uint8, device=dev)
        npairs = C.c_int64(0)
        ps = proj.struct()
        st = lib.gut_bin(L.ref(ps), n, arr, nc, L.ref(p), _ptr(ws), ws.numel(), ids.shape[0],
                         _ptr(ranges), _ptr(ids), C.byref(npairs), _stream())
        if st == L.GUT_E_CAPACITY:
            cap = int(npairs.value * 1.25) + 1024
            ids = None
            continue
        L.check(st, "gut_bin")
        return Bins(ranges=ranges, ids=ids, n_pairs=int(npairs.value), order=order, workspace=ws)
    raise RuntimeError("gut_bin: pair capacity did not converge")


def alloc_image(cams, device="cuda", with_eval=False) -> Image:
    P = num_pixels(cams)
    return Image(rgb=torch.empty(P, 3, device=device), T=torch.empty(P, device=device),
                 n_contrib=torch.empty(P, dtype=torch.int32, device=device),
                 n_eval=torch.empty(P, dtype=torch.int32, device=device) if with_eval else None,
                 shapes=[(int(c["height"]), int(c["width"])) for c in cams])


def _clip_arg(clip, cams):
    """Per-pixel clip distances (hybrid rendering, Sec. 6.2): a float32 device
    tensor with one value per pixel of the call, or None."""
    if clip is None:
        return None
    clip = clip.contiguous()
    if clip.dtype != torch.float32 or clip.numel() != num_pixels(cams) or not clip.is_cuda:
        raise ValueError("clip must be a float32 CUDA tensor with one value per pixel")
    return clip


def render(proj: Projection, bins: Bins, cams, params=None, out: Image | None = None,
           with_eval=False, clip: torch.Tensor | None = None) -> Image:
    if out is None:
        out = alloc_image(cams, proj.depth.device, with_eval)
    arr = L.camera_array(cams)
    p = L.params_struct(params)
    ps = proj.struct()
    clip = _clip_arg(clip, cams)
    L.check(L.load().gut_render(L.ref(ps), proj.n, _ptr(bins.ranges), _ptr(bins.ids), arr,
                                len(cams), L.ref(p), _ptr(clip), _ptr(out.rgb), _ptr(out.T),
                                _ptr(out.n_contrib), _ptr(out.n_eval), _stream()), "gut_render")
    return out


def render_backward(scene: GaussianScene, proj: Projection, bins: Bins, cams, image: Image,
                    d_rgb: torch.Tensor, d_T: torch.Tensor | None = None, params=None,
                    grads: dict | None = None, workspace: torch.Tensor | None = None,
                    clip: torch.Tensor | None = None) -> dict:
    lib = L.load()
    n, nc = scene.n, len(cams)
    dev = scene.means.device
    if grads is None:
        grads = dict(means=torch.empty_like(scene.means), scales=torch.empty_like(scene.scales),
                     quats=torch.empty_like(scene.quats),
                     opacities=torch.empty_like(scene.opacities), sh=torch.empty_like(scene.sh))
    need = lib.gut_render_bwd_workspace_bytes(n, nc)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(int(need), 256), dtype=torch.uint8, device=dev)
    arr = L.camera_array(cams)
    p = L.params_struct(params)
    ss, ps = scene.struct(), proj.struct()
    d_rgb = d_rgb.contiguous()
    d_T = None if d_T is None else d_T.contiguous()
    clip = _clip_arg(clip, cams)
    L.check(lib.gut_render_bwd(L.ref(ss), L.ref(ps), _ptr(bins.ranges), _ptr(bins.ids), arr, nc,
                               L.ref(p), _ptr(clip), _ptr(image.rgb), _ptr(image.T), _ptr(image.n_contrib),
                               _ptr(d_rgb), _ptr(d_T), _ptr(grads["means"]),
                               _ptr(grads["scales"]), _ptr(grads["quats"]),
                               _ptr(grads["opacities"]), _ptr(grads["sh"]), _ptr(workspace),
                               workspace.numel(), _stream()), "gut_render_bwd")
    return grads


def forward(scene: GaussianScene, cams, params=None, with_eval=False, clip=None):
    """project -> bin -> render; returns (proj, bins, image)."""
    proj = project(scene, cams, params)
    bins = bin_tiles(proj, cams, params)
    img = render(proj, bins, cams, params, with_eval=with_eval, clip=clip)
    return proj, bins, img


class GutRender(torch.autograd.Function):
    """Differentiable render of activated particle parameters.

    forward keeps only the compositing state the backward recomputes from
    (T_final, n_contrib, the tile lists and the projected records); with
    ``recompute_projection`` it drops the projection too and re-runs it in
    backward (saves C*n*28 B + n*64 B).  ``clip``: per-pixel clip distances
    of hybrid rendering (Sec. 6.2), used by forward and backward alike."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacities, sh, sh_degree, cams, params,
                recompute_projection, clip=None):
        scene = GaussianScene(means.contiguous(), scales.contiguous(), quats.contiguous(),
                              opacities.contiguous(), sh.contiguous(), int(sh_degree))
        proj, bins, img = forward(scene, cams, params, clip=clip)
        ctx.cams, ctx.params, ctx.sh_degree, ctx.clip = cams, params, int(sh_degree), clip
        ctx.recompute = bool(recompute_projection)
        ctx.bins = bins
        ctx.shapes = img.shapes
        ctx.proj = None if ctx.recompute else proj
        # the outputs go through save_for_backward, so that an in-place edit of
        # a returned image is caught by autograd's version check instead of
        # silently changing the gradients
        ctx.save_for_backward(scene.means, scene.scales, scene.quats, scene.opacities, scene.sh,
                              img.rgb, img.T, img.n_contrib)
        return img.rgb, img.T

    @staticmethod
    def backward(ctx, d_rgb, d_T):
        means, scales, quats, opacities, sh, rgb, T, n_contrib = ctx.saved_tensors
        scene = GaussianScene(means, scales, quats, opacities, sh, ctx.sh_degree)
        img = Image(rgb=rgb, T=T, n_contrib=n_contrib, n_eval=None, shapes=ctx.shapes)
        proj = ctx.proj if ctx.proj is not None else project(scene, ctx.cams, ctx.params)
        if d_rgb is None:
            d_rgb = torch.zeros_like(rgb)
        g = render_backward(scene, proj, ctx.bins, ctx.cams, img, d_rgb, d_T, ctx.params,
                            clip=ctx.clip)
        return g["means"], g["scales"], g["quats"], g["opacities"], g["sh"], None, None, None, None, None


def render_gaussians(means, scales, quats, opacities, sh, sh_degree, cams, params=None,
                     recompute_projection=False, clip=None):
    """Differentiable render; returns (list of [H,W,3] images, list of [H,W] T_final).
    params may select the generalized response (kernel_degree); clip gives
    per-pixel clip distances (hybrid rendering)."""
    rgb, T = GutRender.apply(means, scales, quats, opacities, sh, sh_degree, cams, params,
                             recompute_projection, clip)
    out_rgb, out_T, o = [], [], 0
    for c in cams:
        h, w = int(c["height"]), int(c["width"])
        out_rgb.append(rgb[o:o + h * w].view(h, w, 3))
        out_T.append(T[o:o + h * w].view(h, w))
        o += h * w
    return out_rgb, out_T
