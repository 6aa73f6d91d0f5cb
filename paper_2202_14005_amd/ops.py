"""Thin Python binding of the mrx C-ABI (argument marshalling only).

Every computation runs in the HIP kernels of libmrx.so; torch supplies device
memory, the current stream and, in ``autograd``, the tape.  Complex tensors
are complex64 (interleaved float pairs), contiguous, on one CUDA/HIP device.

Shapes for an even batch: images [B, H, W], coil data [B, C, H, W],
masks [B, H] float32.  For uneven batches (different H, W, C per slice) pass
flat packed 1-D tensors in the layout described in include/mrx.h.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import torch

from ._lib import check, lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """Shapes of a batch of slices plus the library's plan and workspace.

    ``H``, ``W``, ``C`` are ints (even batch of ``B`` slices) or per-slice
    sequences (uneven batch)."""

    def __init__(self, H, W, C, B: int | None = None, device=None, network: bool = False, vn: bool = False,
                 soft: bool = False, toeplitz: bool = False, batchnorm: bool = False):
        L = lib()
        if isinstance(H, int):
            if B is None:
                raise ValueError("B is required for an even batch")
            Hs, Ws, Cs = [H] * B, [W] * B, [C] * B
        else:
            Hs, Ws, Cs = list(H), list(W), list(C)
        self.B = len(Hs)
        self.H, self.W, self.C = Hs, Ws, Cs
        self.even = len(set(zip(Hs, Ws, Cs))) == 1
        self.device = (torch.device(device) if device is not None
                       else torch.device("cuda", torch.cuda.current_device()))
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        arr = lambda v: (ctypes.c_int32 * len(v))(*v)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            flags = ((1 if network else 0) | (2 if vn else 0) | (4 if soft else 0) | (8 if toeplitz else 0)
                     | (16 if batchnorm else 0))
            check(L.mrx_plan_create(ctypes.byref(h), self.B, arr(Hs), arr(Ws), arr(Cs), flags), "plan_create")
        self.network = network
        self.vn = vn
        self.soft = soft
        self.toeplitz = toeplitz
        self.batchnorm = batchnorm
        self._bn = None
        self._weights_key = None
        self._h = h
        ni, nc, nm = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(L.mrx_plan_sizes(h, ctypes.byref(ni), ctypes.byref(nc), ctypes.byref(nm)), "plan_sizes")
        self.n_image, self.n_coil, self.n_mask = ni.value, nc.value, nm.value
        nbytes = int(L.mrx_plan_workspace_bytes(h))
        self.workspace = torch.empty(max(nbytes, 256) + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        with torch.cuda.device(self.device):
            check(L.mrx_plan_set_workspace(h, ctypes.c_void_p(self.workspace.data_ptr() + off), nbytes),
                  "plan_set_workspace")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().mrx_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    # ------------------------------------------------------------ checking
    def _img(self, t, name):
        return self._chk(t, name, self.n_image, torch.complex64, (self.B, self.H[0], self.W[0]))

    def _coil(self, t, name):
        return self._chk(t, name, self.n_coil, torch.complex64, (self.B, self.C[0], self.H[0], self.W[0]))

    def _mask(self, t, name):
        """The sampling argument: the row mask, or on a Toeplitz plan the PSF
        spectrum (float32 [B, 2H, 2W])."""
        if self.toeplitz:
            return self._chk(t, name, 4 * self.n_image, torch.float32, (self.B, 2 * self.H[0], 2 * self.W[0]))
        return self._chk(t, name, self.n_mask, torch.float32, (self.B, self.H[0]))

    # ------------------------------------------------------ non-Cartesian
    def _traj(self, traj):
        if not isinstance(traj, torch.Tensor) or traj.dtype != torch.float32 or not traj.is_contiguous():
            raise TypeError("traj must be a contiguous float32 tensor [B, M, 2]")
        if traj.dim() != 3 or traj.shape[0] != self.B or traj.shape[2] != 2:
            raise ValueError(f"traj must have shape [B, M, 2], got {tuple(traj.shape)}")
        return int(traj.shape[1])

    def nufft_fwd(self, x, S, traj, noise=None, out=None):
        """y = A x (+ noise): the non-uniform DFT of the coil images at the
        trajectory, complex64 [B, C, M] (even batch; packed otherwise)."""
        M = self._traj(traj)
        self._img(x, "x"); self._coil(S, "S")
        n = sum(self.C) * M
        y = out if out is not None else torch.empty(
            (self.B, self.C[0], M) if self.even else (n,), dtype=torch.complex64, device=self.device)
        for t, nm in ((y, "out"), (noise, "noise")):
            if t is not None and (t.dtype != torch.complex64 or t.numel() != n or not t.is_contiguous()):
                raise ValueError(f"{nm} must be a contiguous complex64 tensor of {n} elements")
        check(lib().mrx_nufft_fwd(self._h, _ptr(traj), M, _ptr(x), _ptr(S), _ptr(noise), _ptr(y),
                                  _stream(self.device)), "nufft_fwd")
        return y

    def nufft_adj(self, y, S, traj, out=None):
        """x = A^H y, the adjoint reconstruction from non-Cartesian data."""
        M = self._traj(traj)
        self._coil(S, "S")
        if y.dtype != torch.complex64 or y.numel() != sum(self.C) * M or not y.is_contiguous():
            raise ValueError("y must be a contiguous complex64 tensor of sum(C) * M elements")
        x = self._img(out, "out") if out is not None else self._empty_img()
        check(lib().mrx_nufft_adj(self._h, _ptr(traj), M, _ptr(y), _ptr(S), _ptr(x), _stream(self.device)),
              "nufft_adj")
        return x

    def toeplitz_psf(self, traj, out=None):
        """The real PSF spectrum on the twice-padded grid, float32 [B, 2H, 2W]."""
        M = self._traj(traj)
        shape = (self.B, 2 * self.H[0], 2 * self.W[0]) if self.even else (4 * self.n_image,)
        o = out if out is not None else torch.empty(shape, dtype=torch.float32, device=self.device)
        self._chk(o, "out", 4 * self.n_image, torch.float32, (self.B, 2 * self.H[0], 2 * self.W[0]))
        check(lib().mrx_toeplitz_psf(self._h, _ptr(traj), M, _ptr(o), _stream(self.device)), "toeplitz_psf")
        return o

    def _chk(self, t, name, numel, dtype, even_shape):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if t.device != self.device and not (t.device.type == "cuda" and self.device.type == "cuda"
                                             and t.device.index == self.device.index):
            raise ValueError(f"{name} must be on {self.device}, got {t.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, plan needs {numel}")
        if self.even and t.dim() > 1 and tuple(t.shape) != even_shape:
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {even_shape}")
        return t

    def lam(self, lam):
        """Per-slice lambda as a device float32 tensor [B]."""
        if isinstance(lam, torch.Tensor):
            t = lam.to(device=self.device, dtype=torch.float32).reshape(-1)
            if t.numel() == 1:
                t = t.expand(self.B)
            return t.contiguous()
        if isinstance(lam, (int, float)):
            return torch.full((self.B,), float(lam), dtype=torch.float32, device=self.device)
        return torch.tensor(list(lam), dtype=torch.float32, device=self.device)

    def _empty_img(self):
        shape = (self.B, self.H[0], self.W[0]) if self.even else (self.n_image,)
        return torch.empty(shape, dtype=torch.complex64, device=self.device)

    def _empty_coil(self):
        shape = (self.B, self.C[0], self.H[0], self.W[0]) if self.even else (self.n_coil,)
        return torch.empty(shape, dtype=torch.complex64, device=self.device)

    # ----------------------------------------------------------- operators
    def sense_fwd(self, x, S, mask, noise=None, out=None):
        """y = mask * (F(S x) + noise)."""
        self._img(x, "x"); self._coil(S, "S"); self._mask(mask, "mask"); self._coil(noise, "noise")
        y = self._coil(out, "out") if out is not None else self._empty_coil()
        check(lib().mrx_sense_fwd(self._h, _ptr(x), _ptr(S), _ptr(mask), _ptr(noise), _ptr(y),
                                  _stream(self.device)), "sense_fwd")
        return y

    def sense_adj(self, y, S, mask, out=None):
        """x = sum_c conj(S_c) F^H(mask * y_c)."""
        self._coil(y, "y"); self._coil(S, "S"); self._mask(mask, "mask")
        x = self._img(out, "out") if out is not None else self._empty_img()
        check(lib().mrx_sense_adj(self._h, _ptr(y), _ptr(S), _ptr(mask), _ptr(x), _stream(self.device)),
              "sense_adj")
        return x

    def sense_normal(self, x, S, mask, lam=None, out=None):
        """(A^H A + lambda I) x."""
        self._img(x, "x"); self._coil(S, "S"); self._mask(mask, "mask")
        lt = self.lam(lam) if lam is not None else None
        q = self._img(out, "out") if out is not None else self._empty_img()
        check(lib().mrx_sense_normal(self._h, _ptr(x), _ptr(S), _ptr(mask), _ptr(lt), _ptr(q),
                                     _stream(self.device)), "sense_normal")
        return q

    def cg_dc(self, aHy, S, mask, lam, n_iter, z=None, out=None, hist=False):
        """x = (A^H A + lambda I)^{-1}(aHy + lambda z) by n_iter CG steps from 0.
        With hist=True also returns ||r_k||^2, float32 [B, n_iter + 1]."""
        self._img(aHy, "aHy"); self._img(z, "z"); self._coil(S, "S"); self._mask(mask, "mask")
        lt = self.lam(lam)
        x = self._img(out, "out") if out is not None else self._empty_img()
        h = torch.empty((self.B, n_iter + 1), dtype=torch.float32, device=self.device) if hist else None
        check(lib().mrx_cg_dc(self._h, _ptr(aHy), _ptr(z), _ptr(S), _ptr(mask), _ptr(lt), int(n_iter),
                              _ptr(x), _ptr(h), _stream(self.device)), "cg_dc")
        return (x, h) if hist else x

    def cg_dc_noalloc(self, aHy, S, mask, lam, n_iter, z=None, out=None, hist=False, flags=None):
        """cg_dc through the library's allocation-free entry point (fixed
        device scratch instead of the plan workspace).  ``out``, ``hist`` and
        ``flags`` (uint32 [B], this call's status bits) may be passed
        preallocated so that the call itself allocates nothing."""
        self._img(aHy, "aHy"); self._img(z, "z"); self._coil(S, "S"); self._mask(mask, "mask")
        lt = self.lam(lam)
        x = self._img(out, "out") if out is not None else self._empty_img()
        h = hist if isinstance(hist, torch.Tensor) else (
            torch.empty((self.B, n_iter + 1), dtype=torch.float32, device=self.device) if hist else None)
        check(lib().mrx_cg_dc_noalloc(self._h, _ptr(aHy), _ptr(z), _ptr(S), _ptr(mask), _ptr(lt), int(n_iter),
                                      _ptr(x), _ptr(h), _ptr(flags), _stream(self.device)), "cg_dc_noalloc")
        return (x, h) if h is not None else x

    def cg_dc_backward(self, gx, x, S, mask, lam, n_iter, z=None, need_z=True, need_lam=True):
        """Returns (g_aHy, g_z or None, g_lambda [B] or None)."""
        self._img(gx, "gx"); self._img(x, "x"); self._img(z, "z"); self._coil(S, "S"); self._mask(mask, "mask")
        lt = self.lam(lam)
        ga = self._empty_img()
        gz = self._empty_img() if need_z else None
        gl = torch.zeros(self.B, dtype=torch.float32, device=self.device) if need_lam else None
        check(lib().mrx_cg_dc_backward(self._h, _ptr(gx), _ptr(x), _ptr(z), _ptr(S), _ptr(mask), _ptr(lt),
                                       int(n_iter), _ptr(ga), _ptr(gz), _ptr(gl), 0,
                                       _stream(self.device)), "cg_dc_backward")
        return ga, gz, gl

    def dc_judge(self, x_net, x_cg, aHy, S, mask, ratio, out=None, choice=None):
        """Per slice keep x_net unless it is non-finite, flagged, or its
        residual ||A^H A x - aHy|| exceeds ratio times that of the CG-SENSE
        result x_cg.  Returns (out, choice int32 [B]: 1 = fallback taken)."""
        self._img(x_net, "x_net"); self._img(x_cg, "x_cg"); self._img(aHy, "aHy")
        self._coil(S, "S"); self._mask(mask, "mask")
        o = self._img(out, "out") if out is not None else self._empty_img()
        if choice is None:
            choice = torch.empty(self.B, dtype=torch.int32, device=self.device)
        elif choice.dtype != torch.int32 or choice.numel() != self.B or not choice.is_contiguous():
            raise ValueError("choice must be a contiguous int32 tensor [B]")
        check(lib().mrx_dc_judge(self._h, _ptr(x_net), _ptr(x_cg), _ptr(aHy), _ptr(S), _ptr(mask), float(ratio),
                                 _ptr(o), _ptr(choice), _stream(self.device)), "dc_judge")
        return o, choice

    def status(self, clear=False, out=None):
        """Per-slice status bits (uint32 words in an int32 tensor [B] on the device)."""
        f = torch.zeros(self.B, dtype=torch.int32, device=self.device) if out is None else out
        if f.dtype != torch.int32 or f.numel() != self.B or not f.is_contiguous() or f.device != self.device:
            raise ValueError("out must be a contiguous int32 tensor [B] on the plan's device")
        check(lib().mrx_status_word(self._h, _ptr(f), int(bool(clear)), _stream(self.device)), "status_word")
        return f

    def clear_status(self):
        """Reset the per-slice status words (enqueued; no copy)."""
        check(lib().mrx_status_word(self._h, None, 1, _stream(self.device)), "status_word")

    def autotune(self, S, mask):
        a = self._empty_img().normal_()
        b = self._empty_img()
        check(lib().mrx_plan_autotune(self._h, _ptr(S), _ptr(mask), _ptr(a), _ptr(b), _stream(self.device)),
              "autotune")

    def schedule(self, b=0):
        return lib().mrx_plan_schedule(self._h, int(b)).decode()

    # kernel ids of kernel_time
    KERNEL_NORMAL, KERNEL_CG_UPDATE, KERNEL_CONV_MID, KERNEL_WGRAD_MID = 0, 1, 2, 3
    KERNEL_VN_FILTER, KERNEL_VN_FILTER_REV, KERNEL_VN_ADJOINT, KERNEL_VN_KGRAD = 4, 5, 6, 7

    def kernel_timing(self, enable: bool):
        """Switch per-launch event timing of the hot kernels on or off (and
        drop the records so far)."""
        check(lib().mrx_plan_kernel_timing(self._h, int(bool(enable))), "kernel_timing")

    def kernel_time(self, kid: int):
        """(summed microseconds, launches) of kernel ``kid`` since timing was
        switched on; synchronises with the recorded launches."""
        t, n = ctypes.c_double(0.0), ctypes.c_int32(0)
        check(lib().mrx_plan_kernel_time(self._h, int(kid), ctypes.byref(t), ctypes.byref(n)), "kernel_time")
        return t.value, n.value

    def set_schedule(self, n, name):
        check(lib().mrx_plan_set_schedule(self._h, int(n), name.encode()), "plan_set_schedule")


    # ------------------------------------------------------------- network
    def set_bn(self, bn: "BatchNorm"):
        """Batch normalisation parameters for every later network call (plan
        created with batchnorm=True); the tensors are kept referenced."""
        if not self.batchnorm:
            raise ValueError("set_bn needs a plan created with batchnorm=True")
        check(lib().mrx_cnn_set_bn(self._h, _ptr(bn.gamma), _ptr(bn.beta), _ptr(bn.g_gamma), _ptr(bn.g_beta)),
              "cnn_set_bn")
        self._bn = bn

    def set_weights(self, cnn: "CNN", force=False):
        """Pack the denoiser weights (bf16 MFMA fragments) into the workspace;
        skipped when the same weights (same tensors and version) are packed."""
        key = cnn.key()
        if force or key != self._weights_key:
            check(lib().mrx_cnn_set_weights(self._h, ctypes.byref(cnn.c_params()), _stream(self.device)),
                  "cnn_set_weights")
            self._weights_key = key

    def cnn_forward(self, x, cnn: "CNN", out=None):
        """z = x + N(x)."""
        self._img(x, "x")
        self.set_weights(cnn)
        z = self._img(out, "out") if out is not None else self._empty_img()
        check(lib().mrx_cnn_forward(self._h, _ptr(x), _ptr(z), _stream(self.device)), "cnn_forward")
        return z

    def cnn_layer_forward(self, layer, a_in, cnn: "CNN", out=None):
        """One 64-channel layer on bf16 NHWC activations (torch.bfloat16
        tensors of n_image * 64 elements)."""
        self.set_weights(cnn)
        if a_in.dtype != torch.bfloat16 or a_in.numel() != self.n_image * 64 or not a_in.is_contiguous():
            raise ValueError("a_in must be a contiguous bfloat16 tensor of n_image * 64 elements")
        out = torch.empty_like(a_in) if out is None else out
        check(lib().mrx_cnn_layer_forward(self._h, int(layer), _ptr(a_in), _ptr(out), _stream(self.device)),
              "cnn_layer_forward")
        return out

    def cnn_backward(self, x, gz, cnn: "CNN", grads: "CNNGrads", accumulate=False):
        """Returns gx = gz + J_N(x)^T gz; weight gradients into grads."""
        self._img(x, "x"); self._img(gz, "gz")
        self.set_weights(cnn)
        gx = self._empty_img()
        check(lib().mrx_cnn_backward(self._h, _ptr(x), _ptr(gz), _ptr(gx), ctypes.byref(grads.c_grads()),
                                     int(bool(accumulate)), _stream(self.device)), "cnn_backward")
        return gx

    def modl_forward(self, aHy, S, mask, cnn: "CNN", lam, T, n_cg, states=False, out=None, x0=None):
        """x^T of eq. update_modl from x^0 = aHy (or from ``x0``, as the
        non-Cartesian networks start from a SENSE reconstruction); with
        states=True also the iterates x^0..x^T [T + 1, ...]."""
        self._img(aHy, "aHy"); self._coil(S, "S"); self._mask(mask, "mask"); self._img(x0, "x0")
        self.set_weights(cnn)
        lt = self.lam(lam)
        x = self._img(out, "out") if out is not None else self._empty_img()
        st = (torch.empty((T + 1,) + tuple(x.shape), dtype=torch.complex64, device=self.device)
              if states else None)
        if x0 is None:
            check(lib().mrx_modl_forward(self._h, _ptr(aHy), _ptr(S), _ptr(mask), _ptr(lt), int(T), int(n_cg),
                                         _ptr(x), _ptr(st), _stream(self.device)), "modl_forward")
        else:
            check(lib().mrx_modl_forward_from(self._h, _ptr(x0), _ptr(aHy), _ptr(S), _ptr(mask), _ptr(lt), int(T),
                                              int(n_cg), _ptr(x), _ptr(st), _stream(self.device)), "modl_forward")
        return (x, st) if states else x

    def modl_backward(self, g_out, states, aHy, S, mask, cnn: "CNN", lam, T, n_cg, grads: "CNNGrads",
                      accumulate=False, need_aHy=False):
        """Returns (g_lambda [B], g_aHy or None); weight gradients into grads."""
        self._img(g_out, "g_out"); self._img(aHy, "aHy"); self._coil(S, "S"); self._mask(mask, "mask")
        self.set_weights(cnn)
        lt = self.lam(lam)
        gl = torch.zeros(self.B, dtype=torch.float32, device=self.device)
        ga = self._empty_img() if need_aHy else None
        check(lib().mrx_modl_backward(self._h, _ptr(g_out), _ptr(states), _ptr(aHy), _ptr(S), _ptr(mask),
                                      _ptr(lt), int(T), int(n_cg), ctypes.byref(grads.c_grads()), _ptr(gl),
                                      _ptr(ga), int(bool(accumulate)), _stream(self.device)), "modl_backward")
        return gl, ga

    # ---------------------------------------------------------- soft-SENSE
    # Two coil-map sets: images [B, 2, H, W] (flat 2 n_image for uneven
    # batches), maps [B, 2, C, H, W] (flat 2 n_coil), k-space as for SENSE.
    def _simg(self, t, name):
        return self._chk(t, name, 2 * self.n_image, torch.complex64, (self.B, 2, self.H[0], self.W[0]))

    def _smaps(self, t, name):
        return self._chk(t, name, 2 * self.n_coil, torch.complex64, (self.B, 2, self.C[0], self.H[0], self.W[0]))

    def _empty_simg(self):
        shape = (self.B, 2, self.H[0], self.W[0]) if self.even else (2 * self.n_image,)
        return torch.empty(shape, dtype=torch.complex64, device=self.device)

    def _need_soft(self):
        if not self.soft:
            raise ValueError("this plan was created without soft=True")

    def soft_sense_fwd(self, x, S, mask, noise=None, out=None):
        self._need_soft(); self._simg(x, "x"); self._smaps(S, "S"); self._mask(mask, "mask")
        self._coil(noise, "noise")
        y = self._coil(out, "out") if out is not None else self._empty_coil()
        check(lib().mrx_soft_sense_fwd(self._h, _ptr(x), _ptr(S), _ptr(mask), _ptr(noise), _ptr(y),
                                       _stream(self.device)), "soft_sense_fwd")
        return y

    def soft_sense_adj(self, y, S, mask, out=None):
        self._need_soft(); self._coil(y, "y"); self._smaps(S, "S"); self._mask(mask, "mask")
        x = self._simg(out, "out") if out is not None else self._empty_simg()
        check(lib().mrx_soft_sense_adj(self._h, _ptr(y), _ptr(S), _ptr(mask), _ptr(x), _stream(self.device)),
              "soft_sense_adj")
        return x

    def soft_sense_normal(self, x, S, mask, lam=None, out=None):
        self._need_soft(); self._simg(x, "x"); self._smaps(S, "S"); self._mask(mask, "mask")
        lt = self.lam(lam) if lam is not None else None
        q = self._simg(out, "out") if out is not None else self._empty_simg()
        check(lib().mrx_soft_sense_normal(self._h, _ptr(x), _ptr(S), _ptr(mask), _ptr(lt), _ptr(q),
                                          _stream(self.device)), "soft_sense_normal")
        return q

    def soft_cg_dc(self, aHy, S, mask, lam, n_iter, z=None, out=None, hist=False):
        self._need_soft(); self._simg(aHy, "aHy"); self._simg(z, "z"); self._smaps(S, "S"); self._mask(mask, "mask")
        lt = self.lam(lam)
        x = self._simg(out, "out") if out is not None else self._empty_simg()
        h = torch.empty((self.B, n_iter + 1), dtype=torch.float32, device=self.device) if hist else None
        check(lib().mrx_soft_cg_dc(self._h, _ptr(aHy), _ptr(z), _ptr(S), _ptr(mask), _ptr(lt), int(n_iter),
                                   _ptr(x), _ptr(h), _stream(self.device)), "soft_cg_dc")
        return (x, h) if hist else x

    def soft_modl_forward(self, aHy, S, mask, cnn: "CNN", lam, T, n_cg, states=False, out=None):
        self._need_soft(); self._simg(aHy, "aHy"); self._smaps(S, "S"); self._mask(mask, "mask")
        self.set_weights(cnn)
        lt = self.lam(lam)
        x = self._simg(out, "out") if out is not None else self._empty_simg()
        st = (torch.empty((T + 1,) + tuple(x.shape), dtype=torch.complex64, device=self.device)
              if states else None)
        check(lib().mrx_soft_modl_forward(self._h, _ptr(aHy), _ptr(S), _ptr(mask), _ptr(lt), int(T), int(n_cg),
                                          _ptr(x), _ptr(st), _stream(self.device)), "soft_modl_forward")
        return (x, st) if states else x

    def soft_modl_backward(self, g_out, states, aHy, S, mask, cnn: "CNN", lam, T, n_cg, grads: "CNNGrads",
                           accumulate=False, need_aHy=False):
        self._need_soft(); self._simg(g_out, "g_out"); self._simg(aHy, "aHy"); self._smaps(S, "S")
        self._mask(mask, "mask")
        self.set_weights(cnn)
        lt = self.lam(lam)
        gl = torch.zeros(self.B, dtype=torch.float32, device=self.device)
        ga = self._empty_simg() if need_aHy else None
        check(lib().mrx_soft_modl_backward(self._h, _ptr(g_out), _ptr(states), _ptr(aHy), _ptr(S), _ptr(mask),
                                           _ptr(lt), int(T), int(n_cg), ctypes.byref(grads.c_grads()), _ptr(gl),
                                           _ptr(ga), int(bool(accumulate)), _stream(self.device)),
              "soft_modl_backward")
        return gl, ga

    def soft_coil_mse_grad(self, x, S, ref):
        """(loss [1], g) of the MSE on the coil images against ref (coil sized)."""
        self._need_soft(); self._simg(x, "x"); self._smaps(S, "S"); self._coil(ref, "ref")
        g = self._empty_simg()
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        check(lib().mrx_soft_coil_mse_grad(self._h, _ptr(x), _ptr(S), _ptr(ref), _ptr(g), _ptr(loss),
                                           _stream(self.device)), "soft_coil_mse_grad")
        return loss, g

    def normalize_max(self, x, y=None, ref=None):
        """Scale each slice so that max|x| = 1 (x, and y and ref if given, in
        place); returns the per-slice factors [B]."""
        self._img(x, "x"); self._coil(y, "y"); self._img(ref, "ref")
        sc = torch.empty(self.B, dtype=torch.float32, device=self.device)
        check(lib().mrx_normalize_max(self._h, _ptr(x), _ptr(y), _ptr(ref), _ptr(sc), _stream(self.device)),
              "normalize_max")
        return sc

    # ------------------------------------------------------------- VarNet
    def _vn_params(self, k, w, lam):
        from ._lib import VnParams
        if k.dtype != torch.complex64 or tuple(k.shape) != (24, 11, 11) or not k.is_contiguous():
            raise ValueError("k must be a contiguous complex64 tensor [24, 11, 11]")
        if w.dtype != torch.float32 or tuple(w.shape) != (24, 31) or not w.is_contiguous():
            raise ValueError("w must be a contiguous float32 tensor [24, 31]")
        if lam.dtype != torch.float32 or lam.numel() != 1:
            raise ValueError("lam must be a float32 tensor with one element")
        for t, n in ((k, "k"), (w, "w"), (lam, "lam")):
            if t.device != self.device:
                raise ValueError(f"{n} must be on {self.device}")
        return VnParams(k.data_ptr(), w.data_ptr(), lam.data_ptr())

    def vn_stage(self, x, aHy, S, mask, k, w, lam, out=None):
        """x' = x - sum_i K_i^T Phi'_i(Re(k_i * x)) - lam (A^H A x - aHy)."""
        self._img(x, "x"); self._img(aHy, "aHy"); self._coil(S, "S"); self._mask(mask, "mask")
        prm = self._vn_params(k, w, lam)
        xn = self._img(out, "out") if out is not None else self._empty_img()
        check(lib().mrx_vn_stage(self._h, _ptr(x), _ptr(aHy), _ptr(S), _ptr(mask), ctypes.byref(prm), _ptr(xn),
                                 _stream(self.device)), "vn_stage")
        return xn

    def vn_stage_backward(self, g, x, aHy, S, mask, k, w, lam, grads=None, accumulate=False):
        """Returns (g_x, (g_k, g_w, g_lam)); gradients written into grads if given."""
        self._img(g, "g"); self._img(x, "x"); self._img(aHy, "aHy"); self._coil(S, "S"); self._mask(mask, "mask")
        prm = self._vn_params(k, w, lam)
        gx = self._empty_img()
        if grads is None:
            grads = (torch.zeros_like(k), torch.zeros_like(w), torch.zeros(1, dtype=torch.float32,
                                                                            device=self.device))
        gk, gw, gl = grads
        check(lib().mrx_vn_stage_backward(self._h, _ptr(g), _ptr(x), _ptr(aHy), _ptr(S), _ptr(mask),
                                          ctypes.byref(prm), _ptr(gx), _ptr(gk), _ptr(gw), _ptr(gl),
                                          int(bool(accumulate)), _stream(self.device)), "vn_stage_backward")
        return gx, grads

    def mse_grad(self, x, ref):
        """Returns (loss as a device float tensor [1], gradient)."""
        self._img(x, "x"); self._img(ref, "ref")
        g = self._empty_img()
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        check(lib().mrx_mse_grad(self._h, _ptr(x), _ptr(ref), _ptr(g), _ptr(loss), _stream(self.device)),
              "mse_grad")
        return loss, g


def _cuda(device):
    return torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())


class CNN:
    """fp32 master weights of the 5-layer 3x3 denoiser (channels 2-64-64-64-64-2),
    W[l] [C_out, C_in, 3, 3] and b[l] [C_out], on the device."""

    CHANNELS = (2, 64, 64, 64, 64, 2)

    def __init__(self, weights, biases):
        self.w = [w.contiguous() for w in weights]
        self.b = [b.contiguous() for b in biases]
        self.version = 0
        self.bn = None  # BatchNorm parameters trained with these weights, if any
        for l, (w, b) in enumerate(zip(self.w, self.b)):
            co, ci = self.CHANNELS[l + 1], self.CHANNELS[l]
            if tuple(w.shape) != (co, ci, 3, 3) or tuple(b.shape) != (co,):
                raise ValueError(f"layer {l}: expected W {(co, ci, 3, 3)} and b {(co,)}")
            if w.dtype != torch.float32 or b.dtype != torch.float32:
                raise TypeError("weights must be float32")

    @classmethod
    def from_numpy(cls, wb, device=None):
        dev = _cuda(device)
        return cls([torch.from_numpy(w).to(dev) for w, _ in wb], [torch.from_numpy(b).to(dev) for _, b in wb])

    @classmethod
    def init(cls, seed=7, device=None, last_scale=1.0):
        from synthetic import cnn_weights
        return cls.from_numpy(cnn_weights(seed, last_scale=last_scale), device)

    def params(self):
        out = []
        for w, b in zip(self.w, self.b):
            out += [w, b]
        return out

    def key(self):
        return (self.version,) + tuple((t.data_ptr(), t._version) for t in self.params())

    def c_params(self):
        from ._lib import CnnParams
        p = CnnParams()
        for l in range(5):
            p.w[l] = self.w[l].data_ptr()
            p.b[l] = self.b[l].data_ptr()
        return p

    def numpy(self):
        return [(w.detach().cpu().numpy(), b.detach().cpu().numpy()) for w, b in zip(self.w, self.b)]

    def save(self, path):
        """Weights and biases as plain float32 arrays w0, b0, ..., w4, b4."""
        import numpy as np
        arrs = {}
        for l, (w, b) in enumerate(self.numpy()):
            arrs[f"w{l}"], arrs[f"b{l}"] = w, b
        np.savez(path, **arrs)

    @classmethod
    def load(cls, path, device=None):
        import numpy as np
        with np.load(path, allow_pickle=False) as f:
            wb = [(f[f"w{l}"].astype(np.float32), f[f"b{l}"].astype(np.float32)) for l in range(5)]
        return cls.from_numpy(wb, device)


class CNNGrads:
    """Gradient buffers shaped like a CNN's parameters."""

    def __init__(self, cnn: CNN):
        self.w = [torch.zeros_like(w) for w in cnn.w]
        self.b = [torch.zeros_like(b) for b in cnn.b]

    def c_grads(self):
        from ._lib import CnnGrads
        g = CnnGrads()
        for l in range(5):
            g.w[l] = self.w[l].data_ptr()
            g.b[l] = self.b[l].data_ptr()
        return g

    def params(self):
        out = []
        for w, b in zip(self.w, self.b):
            out += [w, b]
        return out


class BatchNorm:
    """gamma and beta of the denoiser's batch normalisation (device float32
    [4, 64], one row per hidden layer) and their gradient buffers; set on a
    plan created with batchnorm=True by ``Plan.set_bn``."""

    def __init__(self, device=None, gamma=None, beta=None):
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        f = lambda a, v: (torch.as_tensor(a, dtype=torch.float32).to(dev).reshape(4, 64).contiguous()
                          if a is not None else torch.full((4, 64), v, dtype=torch.float32, device=dev))
        self.gamma, self.beta = f(gamma, 1.0), f(beta, 0.0)
        self.g_gamma = torch.zeros_like(self.gamma)
        self.g_beta = torch.zeros_like(self.beta)

    def params(self):
        return [self.gamma, self.beta]

    def grads(self):
        return [self.g_gamma, self.g_beta]


class Adam:
    """Adam state over a CNN's parameters (and, with ``bn``, the batch
    normalisation's gamma and beta), stepped by the library kernel."""

    def __init__(self, cnn: CNN, lr=1e-4, b1=0.9, b2=0.999, eps=1e-8, bn: "BatchNorm | None" = None):
        self.cnn, self.lr, self.b1, self.b2, self.eps, self.bn = cnn, lr, b1, b2, eps, bn
        ps = cnn.params() + (bn.params() if bn is not None else [])
        self.m = [torch.zeros_like(p) for p in ps]
        self.v = [torch.zeros_like(p) for p in ps]
        self.t = 0

    def step(self, grads: CNNGrads):
        self.t += 1
        stream = _stream(self.cnn.w[0].device)
        ps = self.cnn.params() + (self.bn.params() if self.bn is not None else [])
        gs = grads.params() + (self.bn.grads() if self.bn is not None else [])
        for p, g, m, v in zip(ps, gs, self.m, self.v):
            check(lib().mrx_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), self.lr, self.b1, self.b2,
                                      self.eps, self.t, stream), "adam_step")
        self.cnn.version += 1  # the packed bf16 copies are now stale


class MoDL:
    """MoDL network: x^0 = A^H y, T unrolls of [denoiser, CG data consistency].
    With learn_lam the one shared lambda is a trained parameter (a device
    float32 tensor [1]): train_step sums its per-slice gradients, takes an
    Adam step on it with the weights' optimiser settings and keeps it >= 0."""

    def __init__(self, plan: Plan, cnn: CNN, lam=0.05, T=5, n_cg=10, learn_lam=False, bn: "BatchNorm | None" = None):
        if not plan.network:
            raise ValueError("MoDL needs a plan created with network=True")
        self.plan, self.cnn, self.T, self.n_cg = plan, cnn, T, n_cg
        if bn is not None:
            plan.set_bn(bn)
        self.learn_lam = learn_lam
        if learn_lam:
            self.lam = torch.full((1,), float(lam), dtype=torch.float32, device=plan.device)
            self._lam_m = torch.zeros_like(self.lam)
            self._lam_v = torch.zeros_like(self.lam)
            self._lam_g = torch.zeros_like(self.lam)
            self._lam_steps = 0
        else:
            self.lam = lam

    def forward(self, y, S, mask, states=False):
        aHy = self.plan.sense_adj(y, S, mask)
        return self.plan.modl_forward(aHy, S, mask, self.cnn, self.lam, self.T, self.n_cg, states=states)

    def train_step(self, y, S, mask, x_ref, grads: CNNGrads, opt: Adam):
        """One training step: forward with stored states, MSE loss, reverse
        pass (adjoint CG + recomputed denoiser activations), Adam.
        Returns the loss as a device tensor."""
        p = self.plan
        aHy = p.sense_adj(y, S, mask)
        xT, states = p.modl_forward(aHy, S, mask, self.cnn, self.lam, self.T, self.n_cg, states=True)
        loss, g = p.mse_grad(xT, x_ref)
        gl, _ = p.modl_backward(g, states, aHy, S, mask, self.cnn, self.lam, self.T, self.n_cg, grads)
        opt.step(grads)
        if self.learn_lam:
            st = _stream(p.device)
            check(lib().mrx_sum_f32(_ptr(gl), gl.numel(), _ptr(self._lam_g), 0, st), "sum_f32")
            self._lam_steps += 1
            check(lib().mrx_adam_step(_ptr(self.lam), _ptr(self._lam_g), _ptr(self._lam_m), _ptr(self._lam_v), 1,
                                      opt.lr, opt.b1, opt.b2, opt.eps, self._lam_steps, st), "adam_step")
            check(lib().mrx_vn_project(None, 0, 1, _ptr(self.lam), 1, st), "vn_project")
        return loss


class VarNet:
    """Variational network: x^0 = A^H y, then T stages (eq. update_vn) with
    per-stage filters k [T, 24, 11, 11] complex64, RBF weights w [T, 24, 31]
    and step sizes lam [T] (device tensors)."""

    def __init__(self, plan: Plan, k, w, lam):
        if not plan.vn:
            raise ValueError("VarNet needs a plan created with vn=True")
        self.plan, self.k, self.w, self.lam = plan, k.contiguous(), w.contiguous(), lam.contiguous()
        self.T = k.shape[0]

    @classmethod
    def init(cls, plan: Plan, seed=1, T=10):
        from synthetic import vn_params
        p = vn_params(seed, n_stages=T)
        d = plan.device
        return cls(plan, torch.from_numpy(p["k"]).to(d), torch.from_numpy(p["w"]).to(d),
                   torch.from_numpy(p["lam"]).to(d))

    def params(self):
        return [self.k, self.w, self.lam]

    def forward(self, aHy, S, mask, params=None):
        """Returns (x^T, states [T + 1, ...]); params (k, w, lam) override
        the network's own."""
        k, w, lam = params if params is not None else self.params()
        states = [aHy]
        for t in range(self.T):
            states.append(self.plan.vn_stage(states[-1], aHy, S, mask, k[t], w[t], lam[t:t + 1]))
        return states[-1], states

    def backward(self, g, states, aHy, S, mask, params=None):
        """Reverse pass from the stored states; returns (gk, gw, glam, g_x0)."""
        k, w, lam = params if params is not None else self.params()
        gk, gw = torch.zeros_like(k), torch.zeros_like(w)
        gl = torch.zeros_like(lam)
        for t in range(self.T - 1, -1, -1):
            g, _ = self.plan.vn_stage_backward(g, states[t], aHy, S, mask, k[t], w[t],
                                               lam[t:t + 1], grads=(gk[t], gw[t], gl[t:t + 1]))
        return gk, gw, gl, g


def _floats(t):
    """A device tensor as its fp32 storage (complex as interleaved pairs)."""
    return torch.view_as_real(t).reshape(-1) if t.is_complex() else t.reshape(-1)


class IPALM:
    """iPALM training of a VarNet (the algorithm the paper names for it):
    step k extrapolates y = theta + alpha_k (theta - theta_prev) with
    alpha_k = (k - 1) / (k + 2), takes the MSE gradient of the network at y
    on the given batch, steps theta = y - tau g and projects onto the
    VarNet constraints (filters zero mean and unit norm, step sizes >= 0).
    The projection is applied to the initial weights too."""

    def __init__(self, net: "VarNet", tau: float):
        self.net, self.tau, self.steps = net, float(tau), 0
        st = _stream(net.plan.device)
        T = net.T
        check(lib().mrx_vn_project(_ptr(net.k), T * net.k.shape[1], net.k.shape[2] * net.k.shape[3], _ptr(net.lam), T,
                                   st), "vn_project")
        self.prev = [p.clone() for p in net.params()]
        self.work = [torch.empty_like(p) for p in net.params()]

    def step(self, aHy, S, mask, ref):
        """One iPALM step on the batch (aHy, S, mask) with reference images
        ref; returns the loss at the extrapolated point (device [1])."""
        net, plan = self.net, self.net.plan
        st = _stream(plan.device)
        self.steps += 1
        a = (self.steps - 1.0) / (self.steps + 2.0)
        for th, pr, y in zip(net.params(), self.prev, self.work):
            check(lib().mrx_ipalm_extrapolate(_ptr(th), _ptr(pr), _ptr(y), _floats(th).numel(), a, st),
                  "ipalm_extrapolate")
        x, states = net.forward(aHy, S, mask, params=self.work)
        loss, g = plan.mse_grad(x, ref)
        grads = net.backward(g, states, aHy, S, mask, params=self.work)[:3]
        for th, pr, y, gg in zip(net.params(), self.prev, self.work, grads):
            check(lib().mrx_ipalm_update(_ptr(th), _ptr(pr), _ptr(y), _ptr(gg), _floats(th).numel(), self.tau, st),
                  "ipalm_update")
        T = net.T
        check(lib().mrx_vn_project(_ptr(net.k), T * net.k.shape[1], net.k.shape[2] * net.k.shape[3], _ptr(net.lam), T,
                                   st), "vn_project")
        return loss


def schedules(n: int):
    """Names of the registered column schedules for transform length n."""
    out, i = [], 0
    while True:
        s = lib().mrx_schedule_name(int(n), i)
        if not s:
            return out
        out.append(s.decode())
        i += 1


def tune_cache_save(path: str):
    """Write the schedules chosen by Plan.autotune in this process to a file."""
    check(lib().mrx_tune_cache_save(str(path).encode()), "tune_cache_save")


def tune_cache_load(path: str) -> int:
    """Merge a saved tuning cache; plans created afterwards use it.  Returns
    the number of entries."""
    n = ctypes.c_int32(0)
    check(lib().mrx_tune_cache_load(str(path).encode(), ctypes.byref(n)), "tune_cache_load")
    return n.value


def supported_length(n: int) -> bool:
    return bool(lib().mrx_supported_length(int(n)))
