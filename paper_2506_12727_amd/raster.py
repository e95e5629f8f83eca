"""Torch-facing API over the mvgs C ABI: a Rasterizer holding one library context, frames,
the fused loss, and the autograd.Function that makes the rasterizer differentiable.

PyTorch provides device memory and the HIP stream (torch's current stream); every step of the
forward, loss and backward runs in libmvgs's kernels.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib as L


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


@dataclass
class GaussianTensors:
    """Activated parameters on the GPU: float32, contiguous."""
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    opacities: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @property
    def P(self) -> int:
        return int(self.means.shape[0])

    @staticmethod
    def from_scene(scene, device="cuda") -> "GaussianTensors":
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).to(device).contiguous()
        return GaussianTensors(f(scene.means), f(scene.scales), f(scene.quats), f(scene.opacities).reshape(-1),
                               f(scene.sh), int(scene.sh_degree))

    def check(self):
        P = self.P
        K = (self.sh_degree + 1) ** 2
        shapes = {"means": (P, 3), "scales": (P, 3), "quats": (P, 4), "opacities": (P,), "sh": (P, K, 3)}
        for n, shp in shapes.items():
            t = getattr(self, n)
            if tuple(t.shape) != shp or t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{n}: expected contiguous float32 cuda tensor of shape {shp}, got "
                                 f"{tuple(t.shape)} {t.dtype} on {t.device}")


def _check_grads(g: GaussianTensors, grads: dict):
    for name in ("means", "scales", "quats", "opacities", "sh"):
        t = grads[name]
        if t.shape != getattr(g, name).shape or t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"grads[{name!r}] does not match the Gaussians")


class Frame:
    """Saved forward state (library-owned) for one batch of views."""

    def __init__(self, rast: "Rasterizer", handle: C.c_void_p, cams):
        self.rast, self.handle, self.cams = rast, handle, list(cams)
        self.released = False

    def check(self):
        """Capacity mode: wait for the forward and raise MvgsError if its results are void: records
        or pairs over the context's capacities (MVGS_ECAPACITY), or for a partial frame a rejected
        pixel selection, or a selection of W*H pixels that is no partition of the plane
        (MVGS_EINVAL). No-op otherwise."""
        L.check(L.lib().mvgs_frame_check(self.rast.ctx, _stream(), self.handle), self.rast.ctx)

    def void_word(self) -> Optional[int]:
        """Device address of the word that is non-zero when this capacity-mode frame is void
        (None for other frames)."""
        w = C.c_void_p()
        L.check(L.lib().mvgs_frame_void_word(self.handle, C.byref(w)))
        return w.value

    def set_cameras(self, cams):
        """For a frame made under graph capture: the cameras the next replay renders (same sizes)."""
        L.check(L.lib().mvgs_frame_set_cameras(self.rast.ctx, self.handle, L.camera_array(cams), len(cams)),
                self.rast.ctx)
        self.cams = list(cams)

    def workspace(self) -> int:
        """Device bytes the forward that made this frame asked for (exact sizes)."""
        b = C.c_int64()
        L.check(L.lib().mvgs_frame_workspace(self.handle, C.byref(b)))
        return int(b.value)

    def info(self):
        V, K, T = C.c_int64(), C.c_int64(), C.c_int64()
        L.check(L.lib().mvgs_frame_info(self.handle, C.byref(V), C.byref(K), C.byref(T)))
        dp, tp = C.c_int32(), C.c_int32()
        L.check(L.lib().mvgs_frame_sort_info(self.handle, C.byref(dp), C.byref(tp)))
        return dict(records=V.value, pairs=K.value, tiles=T.value, depth_passes=dp.value, tile_passes=tp.value)

    def release(self):
        if not self.released:
            self.rast.release(self)

    def __del__(self):
        # a frame dropped without release (e.g. an autograd graph freed before its backward)
        # returns its memory to the context, if the context still exists
        try:
            if not self.released and self.rast.ctx:
                self.rast.release(self)
        except Exception:
            pass


class TorchAllocator:
    """Device memory of a library context from PyTorch's caching allocator (mvgs_options.alloc /
    free): blocks are taken on the calling thread's current stream, which is the stream of the
    library call that asks for them, and given back to the cache in that stream's order."""

    def __init__(self, device=None):
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.alloc_fn = L.ALLOC_FN(self._alloc)
        self.free_fn = L.FREE_FN(self._free)

    def _alloc(self, nbytes, _ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), self.device)
        except Exception:   # out of memory: the library returns MVGS_ENOMEM
            return None

    def _free(self, ptr, _ctx):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass


class Rasterizer:
    def __init__(self, tile=(16, 16), pixels_per_lane=0, workspace_limit=0, capacity=None, torch_allocator=True):
        """capacity: None, or (records, pairs) for capacity mode (no host synchronization in the
        forward; capturable into a HIP graph). torch_allocator: the context's workspace and frames
        come from PyTorch's caching allocator (else hipMalloc)."""
        self.lib = L.lib()
        opt = L.mvgs_options()
        opt.tile_w, opt.tile_h = int(tile[0]), int(tile[1])
        opt.pixels_per_lane = int(pixels_per_lane)
        opt.workspace_limit = int(workspace_limit)
        if capacity is not None:
            opt.capacity_records, opt.capacity_pairs = int(capacity[0]), int(capacity[1])
        self.allocator = TorchAllocator() if torch_allocator else None
        if self.allocator is not None:
            opt.alloc, opt.free = self.allocator.alloc_fn, self.allocator.free_fn
        self.capacity = capacity
        self.ctx = C.c_void_p()
        L.check(self.lib.mvgs_create(C.byref(self.ctx), C.byref(opt)))
        self.tile = (opt.tile_w, opt.tile_h)

    def count_views(self, g: GaussianTensors, cams):
        """Participation pre-pass: per view, (participating Gaussians, covered (Gaussian, tile)
        pairs) as int64 arrays; one synchronization of the current stream."""
        import numpy as np
        g.check()
        B = len(cams)
        rec = np.zeros(B, np.int64)
        pairs = np.zeros(B, np.int64)
        L.check(self.lib.mvgs_count_views(self.ctx, _stream(), C.byref(self._gauss(g)), L.camera_array(cams), B,
                                          rec.ctypes.data, pairs.ctypes.data), self.ctx)
        return rec, pairs

    def workspace_bound(self, cams, P: int, records: int, pairs: int, work: int = L.MVGS_WORK_FORWARD) -> int:
        """Device bytes this context would hold after a forward of `cams` (with the loss and backward
        of `work`) whose views count `records` and `pairs` in total (host only)."""
        b = C.c_int64()
        L.check(self.lib.mvgs_workspace_bound(self.ctx, L.camera_array(cams), len(cams), int(P), int(records),
                                              int(pairs), int(work), C.byref(b)), self.ctx)
        return int(b.value)

    def set_workspace_limit(self, nbytes: int):
        """Most device bytes this context may hold from now on (0: no limit)."""
        L.check(self.lib.mvgs_set_workspace_limit(self.ctx, int(nbytes)), self.ctx)

    def memory_held(self) -> int:
        b = C.c_int64()
        L.check(self.lib.mvgs_memory_held(self.ctx, C.byref(b)), self.ctx)
        return int(b.value)

    def close(self):
        if self.ctx:
            self.lib.mvgs_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _gauss(g: GaussianTensors) -> L.mvgs_gaussians:
        s = L.mvgs_gaussians()
        s.P, s.sh_degree = g.P, g.sh_degree
        s.means, s.scales, s.quats = g.means.data_ptr(), g.scales.data_ptr(), g.quats.data_ptr()
        s.opacities, s.sh = g.opacities.data_ptr(), g.sh.data_ptr()
        return s

    def forward(self, g: GaussianTensors, cams, images: Optional[List[torch.Tensor]] = None):
        """Render every view of `cams`; returns ([3,H,W] float32 images, Frame)."""
        g.check()
        dev = g.means.device
        if images is None:
            images = [torch.empty((3, c.height, c.width), dtype=torch.float32, device=dev) for c in cams]
        ca = L.camera_array(cams)
        gs = self._gauss(g)
        fr = C.c_void_p()
        st = self.lib.mvgs_forward(self.ctx, _stream(), C.byref(gs), ca, len(cams),
                                   L.ptr_array([t.data_ptr() for t in images]), C.byref(fr))
        L.check(st, self.ctx)
        return images, Frame(self, fr, cams)

    def subsample(self, cams, keys: torch.Tensor):
        """Alg. 3's index array for views of one size from one random uint32 key per pixel position
        (int32 tensor [H*W] on the GPU holding the key bits): (sel_offsets, sel_pixels) int32 tensors."""
        W, H = int(cams[0].width), int(cams[0].height)
        tiles = ((W + self.tile[0] - 1) // self.tile[0]) * ((H + self.tile[1] - 1) // self.tile[1])
        off = torch.empty(len(cams) * tiles + 1, dtype=torch.int32, device=keys.device)
        pix = torch.empty(W * H, dtype=torch.int32, device=keys.device)
        keys = keys.contiguous()
        L.check(self.lib.mvgs_subsample(self.ctx, _stream(), L.camera_array(cams), len(cams), keys.data_ptr(),
                                        off.data_ptr(), pix.data_ptr()), self.ctx)
        return off, pix

    def forward_partial(self, g: GaussianTensors, cams, sel_offsets: torch.Tensor, sel_pixels: torch.Tensor,
                        mode: int = L.MVGS_PARTIAL_COMPACT, images: Optional[List[torch.Tensor]] = None):
        """Render only the selected pixels (Alg. 3). `images` (default: zero-filled) receive the
        selected pixels; pass the same tensor for every view to get the merged image."""
        g.check()
        dev = g.means.device
        if images is None:
            images = [torch.zeros((3, c.height, c.width), dtype=torch.float32, device=dev) for c in cams]
        sel_offsets, sel_pixels = sel_offsets.contiguous(), sel_pixels.contiguous()
        fr = C.c_void_p()
        st = self.lib.mvgs_forward_partial(self.ctx, _stream(), C.byref(self._gauss(g)), L.camera_array(cams),
                                           len(cams), sel_offsets.data_ptr(), sel_pixels.data_ptr(),
                                           int(sel_pixels.numel()), int(mode),
                                           L.ptr_array([t.data_ptr() for t in images]), C.byref(fr))
        L.check(st, self.ctx)
        return images, Frame(self, fr, cams)

    def loss(self, cams, images, targets, w_l1=1.0, w_dssim=0.0, out=None, grads=None, noalloc=False):
        """Fused L1 + D-SSIM: returns (loss [1] tensor on the GPU, list of dL/dimage). noalloc: through
        mvgs_loss_noalloc (the library's fixed per-GPU scratch; give out and grads to allocate
        nothing here either)."""
        dev = images[0].device
        if out is None:
            out = torch.empty(1, dtype=torch.float32, device=dev)
        if grads is None:
            grads = [torch.empty_like(t) for t in images]
        ca = L.camera_array(cams)
        fn = self.lib.mvgs_loss_noalloc if noalloc else self.lib.mvgs_loss
        st = fn(self.ctx, _stream(), ca, len(cams), L.ptr_array([t.data_ptr() for t in images]),
                L.ptr_array([t.data_ptr() for t in targets]), float(w_l1), float(w_dssim), out.data_ptr(),
                L.ptr_array([t.data_ptr() for t in grads]))
        L.check(st, self.ctx)
        return out, grads

    def backward(self, g: GaussianTensors, frame: Frame, dl_dimages, densify=None, grads=None):
        """Parameter gradients (overwritten) and, if `densify` = dict(e1, e2, count) tensors, the
        densification statistics (accumulated)."""
        if frame.released:
            raise ValueError("the frame was released: render again for another backward")
        g.check()
        if grads is None:
            grads = dict(means=torch.empty_like(g.means), scales=torch.empty_like(g.scales),
                         quats=torch.empty_like(g.quats), opacities=torch.empty_like(g.opacities),
                         sh=torch.empty_like(g.sh))
        gr = self._grads(grads)
        dz = None
        if densify is not None:
            dz = L.mvgs_densify()
            dz.e1, dz.e2, dz.count = densify["e1"].data_ptr(), densify["e2"].data_ptr(), densify["count"].data_ptr()
        gs = self._gauss(g)
        dl = [t.contiguous() for t in dl_dimages]
        st = self.lib.mvgs_backward(self.ctx, _stream(), C.byref(gs), frame.handle,
                                    L.ptr_array([t.data_ptr() for t in dl]), C.byref(gr),
                                    C.byref(dz) if dz is not None else None)
        L.check(st, self.ctx)
        return grads

    def release(self, frame: Frame):
        if not frame.released:
            L.check(self.lib.mvgs_frame_release(self.ctx, frame.handle), self.ctx)
            frame.released = True

    def export_binning(self, frame: Frame):
        """(keys int64 [K] holding the uint64 keys, values int32 [K], ranges int32 [tiles, 2]) on the GPU."""
        info = frame.info()
        dev = torch.device("cuda")
        K, T = max(info["pairs"], 1), max(info["tiles"], 1)
        keys = torch.empty(K, dtype=torch.int64, device=dev)
        vals = torch.empty(K, dtype=torch.int32, device=dev)
        ranges = torch.empty((T, 2), dtype=torch.int32, device=dev)
        L.check(self.lib.mvgs_export_binning(self.ctx, _stream(), frame.handle, keys.data_ptr(), vals.data_ptr(),
                                             ranges.data_ptr()), self.ctx)
        return keys[:info["pairs"]], vals[:info["pairs"]], ranges[:info["tiles"]]

    def loss_3d(self, frame: Frame, image: torch.Tensor, target: torch.Tensor, w_l1=1.0, w_dssim=0.0, out=None,
                grad=None):
        """L1 + 3D distance-aware D-SSIM on the merged plane of a thread-efficient partial frame:
        (loss [1] on the GPU, dL/dimage [3,H,W]). Pass the gradient for every view to backward."""
        if out is None:
            out = torch.empty(1, dtype=torch.float32, device=image.device)
        if grad is None:
            grad = torch.empty_like(image)
        L.check(self.lib.mvgs_loss_3d(self.ctx, _stream(), frame.handle, image.contiguous().data_ptr(),
                                      target.contiguous().data_ptr(), float(w_l1), float(w_dssim), out.data_ptr(),
                                      grad.data_ptr()), self.ctx)
        return out, grad

    def merge(self, frame: Frame, planes, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Per-view [C,H,W] planes merged into the partial frame's image plane (selected pixels of
        each view from that view's plane; others of `out`, zero if it is new, are kept)."""
        planes = [p.contiguous() for p in planes]
        c0 = frame.cams[0]
        if len(planes) != len(frame.cams):
            raise ValueError(f"{len(planes)} planes for {len(frame.cams)} views")
        for p in planes:
            if p.dim() != 3 or tuple(p.shape[1:]) != (c0.height, c0.width) or p.shape[0] != planes[0].shape[0] \
                    or p.dtype != torch.float32 or not p.is_cuda:
                raise ValueError(f"planes: expected float32 cuda [C, {c0.height}, {c0.width}] tensors")
        if out is None:
            out = torch.zeros_like(planes[0])
        elif tuple(out.shape) != tuple(planes[0].shape) or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor shaped like the planes")
        L.check(self.lib.mvgs_frame_merge(self.ctx, _stream(), frame.handle, L.ptr_array([p.data_ptr() for p in planes]),
                                          int(planes[0].shape[0]), out.data_ptr()), self.ctx)
        return out

    def export_depth(self, frame: Frame, outs=None):
        if outs is None:
            outs = [torch.zeros((c.height, c.width), dtype=torch.float32, device="cuda") for c in frame.cams]
        L.check(self.lib.mvgs_export_depth(self.ctx, _stream(), frame.handle,
                                           L.ptr_array([t.data_ptr() for t in outs])), self.ctx)
        return outs

    def adapt_density(self, g: GaussianTensors, stats: dict, normals: torch.Tensor, split_threshold=2e-4,
                clone_threshold=2e-4, dense_scale=0.01, min_opacity=0.005):
        """Multi-view adaptive density control from the statistics dict(e1, e2, count): returns the new
        GaussianTensors and the original index of each new Gaussian (int32). normals: [P, 2, 3]
        standard normal draws for the split children."""
        g.check()
        P = g.P
        K = (g.sh_degree + 1) ** 2
        dev = g.means.device
        for name, dt in (("e1", torch.float32), ("e2", torch.float32), ("count", torch.int32)):
            t = stats[name]
            if tuple(t.shape) != (P,) or t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name}: expected contiguous {dt} cuda tensor of shape ({P},)")
        if tuple(normals.shape) != (P, 2, 3) or normals.dtype != torch.float32 or not normals.is_cuda:
            raise ValueError(f"normals: expected float32 cuda tensor of shape ({P}, 2, 3)")
        cap = max(2 * P, 1)
        out = GaussianTensors(torch.empty((cap, 3), device=dev), torch.empty((cap, 3), device=dev),
                              torch.empty((cap, 4), device=dev), torch.empty(cap, device=dev),
                              torch.empty((cap, K, 3), device=dev), g.sh_degree)
        src = torch.empty(cap, dtype=torch.int32, device=dev)
        prm = L.mvgs_adc_params(float(split_threshold), float(clone_threshold), float(dense_scale), float(min_opacity))
        o = L.mvgs_gaussians_out(out.means.data_ptr(), out.scales.data_ptr(), out.quats.data_ptr(),
                                 out.opacities.data_ptr(), out.sh.data_ptr())
        n = C.c_int64()
        normals = normals.contiguous()
        L.check(self.lib.mvgs_adapt_density(self.ctx, _stream(), C.byref(self._gauss(g)), stats["e1"].data_ptr(),
                                      stats["e2"].data_ptr(), stats["count"].data_ptr(), normals.data_ptr(),
                                      C.byref(prm), C.byref(o), src.data_ptr(), cap, C.byref(n)), self.ctx)
        m = int(n.value)
        res = GaussianTensors(out.means[:m].contiguous(), out.scales[:m].contiguous(), out.quats[:m].contiguous(),
                              out.opacities[:m].contiguous(), out.sh[:m].contiguous(), g.sh_degree)
        return res, src[:m]

    @staticmethod
    def _grads(grads: dict) -> L.mvgs_grads:
        gr = L.mvgs_grads()
        gr.means, gr.scales, gr.quats = grads["means"].data_ptr(), grads["scales"].data_ptr(), grads["quats"].data_ptr()
        gr.opacities, gr.sh = grads["opacities"].data_ptr(), grads["sh"].data_ptr()
        return gr

    def adam_step(self, g: GaussianTensors, grads: dict, moments: torch.Tensor, step: int, lr: dict,
                  beta1=0.9, beta2=0.999, eps=1e-15, step_dev: Optional[torch.Tensor] = None,
                  skip: Optional["Frame"] = None):
        """One in-place Adam step of the activated parameters g (log-scale and opacity-logit
        coordinates for scales and opacities); moments: float32 [P, 11 + 3K, 2], zero at first.
        lr: dict(means, scales, quats, opacities, sh_dc, sh_rest). With step_dev (int32 [1] on the
        GPU) the step number is counted on the device (incremented, then used; `step` is not),
        and with `skip` (a capacity-mode frame) nothing changes when that frame is void: the form
        a captured training step takes."""
        g.check()
        K = (g.sh_degree + 1) ** 2
        _check_grads(g, grads)
        if tuple(moments.shape) != (g.P, 11 + 3 * K, 2) or moments.dtype != torch.float32 or \
                not moments.is_contiguous() or not moments.is_cuda:
            raise ValueError(f"moments: expected float32 {(g.P, 11 + 3 * K, 2)}, got {tuple(moments.shape)}")
        o = L.mvgs_gaussians_out(g.means.data_ptr(), g.scales.data_ptr(), g.quats.data_ptr(), g.opacities.data_ptr(),
                                 g.sh.data_ptr())
        prm = L.mvgs_adam_params(lr["means"], lr["scales"], lr["quats"], lr["opacities"], lr["sh_dc"], lr["sh_rest"],
                                 beta1, beta2, eps, int(step))
        if step_dev is not None:
            if step_dev.dtype != torch.int32 or step_dev.numel() != 1 or not step_dev.is_cuda:
                raise ValueError("step_dev: expected an int32 [1] tensor on the GPU")
            prm.step_dev = step_dev.data_ptr()
        if skip is not None:
            prm.skip_dev = skip.void_word()
        L.check(self.lib.mvgs_adam_step(self.ctx, _stream(), g.P, g.sh_degree, C.byref(o),
                                        C.byref(self._grads(grads)), moments.data_ptr(), C.byref(prm)), self.ctx)

    def gather_rows(self, src: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
        """x[src] for a float32 tensor whose first axis indexes Gaussians, on the GPU."""
        x = x.contiguous()
        n = int(src.numel())
        width = math.prod(int(d) for d in x.shape[1:])
        out = torch.empty((n,) + tuple(x.shape[1:]), dtype=x.dtype, device=x.device)
        if x.dtype != torch.float32 or src.dtype != torch.int32:
            raise ValueError("gather_rows takes float32 rows and int32 indices")
        L.check(self.lib.mvgs_gather_rows(self.ctx, _stream(), src.data_ptr(), n, width, x.data_ptr(),
                                          out.data_ptr()), self.ctx)
        return out

    def grad_moments(self, g: GaussianTensors, grads: dict, sum_: torch.Tensor, acc: torch.Tensor):
        """Adds one mini-batch gradient to the running moments (sum float64 [P (11 + 3K)], acc
        float64 [2]) of the Monte Carlo variance estimate."""
        n = g.P * (11 + 3 * (g.sh_degree + 1) ** 2)
        for t, want in ((sum_, n), (acc, 2)):
            if t.dtype != torch.float64 or t.numel() != want or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"moment buffer: expected contiguous float64 cuda tensor of {want} elements")
        _check_grads(g, grads)
        L.check(self.lib.mvgs_grad_moments(self.ctx, _stream(), g.P, g.sh_degree, C.byref(self._grads(grads)),
                                           sum_.data_ptr(), acc.data_ptr()), self.ctx)

    def export_transmittance(self, frame: Frame, outs=None):
        """Final transmittance [H,W] of each view (of the selected pixels only for a thread-efficient
        partial frame: other pixels of `outs` are kept)."""
        if outs is None:
            outs = [torch.zeros((c.height, c.width), dtype=torch.float32, device="cuda") for c in frame.cams]
        L.check(self.lib.mvgs_export_transmittance(self.ctx, _stream(), frame.handle,
                                                   L.ptr_array([t.data_ptr() for t in outs])), self.ctx)
        return outs


class MVGSRasterize(torch.autograd.Function):
    """images = rasterize(means, scales, quats, opacities, sh) for a fixed camera batch.

    The backward recomputes blend state from the frame's final transmittance and last contributor;
    if `densify` (dict of e1, e2, count tensors) is given, the statistics are accumulated into it.
    Frame lifetime: a forward that no backward can follow (grad mode off, or no parameter requires
    grad) releases its frame at once; otherwise the backward releases it, so one forward takes one
    backward (a second raises), and a graph freed without a backward releases it when the frame
    object is collected. A capacity-mode forward outside graph capture is checked (an overflow
    raises instead of giving background images and zero gradients)."""

    @staticmethod
    def forward(ctx, rast: Rasterizer, cams, sh_degree: int, densify, keep: bool, means, scales, quats, opacities,
                sh):
        g = GaussianTensors(means.contiguous(), scales.contiguous(), quats.contiguous(), opacities.contiguous(),
                            sh.contiguous(), sh_degree)
        images, frame = rast.forward(g, cams)
        if rast.capacity is not None and not torch.cuda.is_current_stream_capturing():
            try:
                frame.check()
            except Exception:
                rast.release(frame)
                raise
        if not keep:
            rast.release(frame)
        ctx.rast, ctx.frame, ctx.sh_degree, ctx.densify = rast, frame, sh_degree, densify
        ctx.save_for_backward(g.means, g.scales, g.quats, g.opacities, g.sh)
        return tuple(images)

    @staticmethod
    def backward(ctx, *grad_images):
        if ctx.frame.released:
            raise RuntimeError("rasterize: this forward's frame was already released (its backward ran once, or "
                               "it was rendered without grad); render again for another backward")
        means, scales, quats, opacities, sh = ctx.saved_tensors
        g = GaussianTensors(means, scales, quats, opacities, sh, ctx.sh_degree)
        dl = [gi.contiguous() if gi is not None else torch.zeros((3, c.height, c.width), device=means.device)
              for gi, c in zip(grad_images, ctx.frame.cams)]
        try:
            grads = ctx.rast.backward(g, ctx.frame, dl, densify=ctx.densify)
        finally:
            ctx.rast.release(ctx.frame)
        return (None, None, None, None, None, grads["means"], grads["scales"], grads["quats"], grads["opacities"],
                grads["sh"])


def rasterize(rast: Rasterizer, cams, g: GaussianTensors, densify=None):
    """Differentiable render of every view of `cams`: a tuple of [3,H,W] images."""
    params = (g.means, g.scales, g.quats, g.opacities, g.sh)
    keep = torch.is_grad_enabled() and any(t.requires_grad for t in params)
    return MVGSRasterize.apply(rast, cams, g.sh_degree, densify, keep, *params)


class FusedLoss(torch.autograd.Function):
    """L = w_l1 L1 + w_dssim D-SSIM over a batch of views, image gradients from the fused kernel."""

    @staticmethod
    def forward(ctx, rast: Rasterizer, cams, targets, w_l1: float, w_dssim: float, *images):
        loss, grads = rast.loss(cams, [i.contiguous() for i in images], targets, w_l1, w_dssim)
        ctx.grads = grads
        return loss[0]

    @staticmethod
    def backward(ctx, gl):
        return (None, None, None, None, None) + tuple(g * gl for g in ctx.grads)


def fused_loss(rast: Rasterizer, cams, images: Sequence[torch.Tensor], targets, w_l1=1.0, w_dssim=0.0):
    return FusedLoss.apply(rast, cams, targets, float(w_l1), float(w_dssim), *images)
