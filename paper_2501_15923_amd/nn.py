"""Python binding of the warm-start network (include/icarus_nn.h).

PyTorch holds the device buffers (workspace, features, targets, outputs);
every operation of the network runs in the HIP kernels of libicarus_hip.so.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi
from ._abi import lib


NnShape = _abi.NnShape


def _check(rc):
    if rc != 0:
        raise _abi.IcarusError(rc, lib().icr_nn_last_error().decode())


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def in_channels(coord):
    """Input features per column: 8 boundary primitives (+ 2 colatitude channels)."""
    return 10 if coord else 8


def full_dims(dims):
    """(n_theta, n_phi, n_r, c1, c2, hidden, phi_lo, phi_hi, coord) from a
    stored dims vector (files written before the colatitude channels hold 8
    entries: coord 0)."""
    d = tuple(int(v) for v in dims)
    return d + (0,) if len(d) == 8 else d


def init_params(n_theta, n_phi, n_r, c1, c2, hidden, phi_lo=-1, phi_hi=1, coord=0, seed=0):
    """Scaled normal weights (variance 1/fan_in), zero biases; the last layer
    starts small so the initial output is close to the radial expansion."""
    rng = np.random.default_rng(seed)
    no = 8 * n_r
    k1 = 3 * (phi_hi - phi_lo + 1) * in_channels(coord)
    parts = []
    for fan_in, fan_out, scale in ((k1, c1, 1.0), (9 * c1, c2, 1.0), (c2, hidden, 1.0),
                                   (hidden, no, 0.1)):
        parts.append(rng.normal(0.0, scale / np.sqrt(fan_in), (fan_in, fan_out)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


class WarmStartNet:
    def __init__(self, n_theta, n_phi, n_r, c1=64, c2=128, hidden=384, batch_max=8,
                 phi_lo=-1, phi_hi=1, coord=0, device=0, stream=None):
        import torch
        self.torch = torch
        self.shape = NnShape(n_theta, n_phi, n_r, c1, c2, hidden, batch_max, phi_lo, phi_hi,
                             coord)
        self.dims = (n_theta, n_phi, n_r, c1, c2, hidden, phi_lo, phi_hi, coord)
        self.cin = in_channels(coord)
        self.device = torch.device("cuda", device)
        n = ctypes.c_longlong()
        _check(lib().icr_nn_param_count(ctypes.byref(self.shape), ctypes.byref(n)))
        self.nparam = n.value
        nb = ctypes.c_size_t()
        _check(lib().icr_nn_workspace_bytes(ctypes.byref(self.shape), ctypes.byref(nb)))
        self._ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._ws.data_ptr() + 255) & ~255
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().icr_nn_create(ctypes.byref(self.shape), ctypes.c_void_p(ptr), nb.value,
                                   ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.ncol = n_theta * n_phi
        self.no = 8 * n_r

    def close(self):
        if getattr(self, "h", None):
            lib().icr_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparam
        _check(lib().icr_nn_set_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self):
        out = np.zeros(self.nparam, dtype=np.float32)
        _check(lib().icr_nn_get_params(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    @classmethod
    def from_dims(cls, dims, batch_max=8, **kw):
        """The network of a stored dims vector (8 or 9 entries)."""
        nt, nph, nr, c1, c2, h, lo, hi, coord = full_dims(dims)
        return cls(nt, nph, nr, c1, c2, h, batch_max=batch_max, phi_lo=lo, phi_hi=hi,
                   coord=coord, **kw)

    def forward(self, x):
        """x: torch float32 [B][nt][np][C] on the device -> y [B*ncol][no]."""
        B = x.shape[0]
        y = self.torch.empty((B * self.ncol, self.no), dtype=self.torch.float32,
                             device=self.device)
        _check(lib().icr_nn_forward(self.h, B, _p(x), _p(y)))
        return y

    def loss_grad(self, x, t, want_grad=False):
        B = x.shape[0]
        loss = ctypes.c_double()
        g = np.zeros(self.nparam, dtype=np.float32) if want_grad else None
        _check(lib().icr_nn_loss_grad(
            self.h, B, _p(x), _p(t), ctypes.byref(loss),
            g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if want_grad else None))
        return (loss.value, g) if want_grad else loss.value

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().icr_nn_adam_step(self.h, lr, beta1, beta2, eps))

    def encode_map(self, maps, thc, omega, r_in):
        """maps: torch float64 [B][8][nt][np] SI on the device; thc: [nt]."""
        B = maps.shape[0]
        x = self.torch.empty((B, self.shape.n_theta, self.shape.n_phi, self.cin),
                             dtype=self.torch.float32, device=self.device)
        _check(lib().icr_nn_encode_map(self.h, B, _abi.dptr(maps.data_ptr()),
                                       _abi.dptr(thc.data_ptr()), omega, r_in, _p(x)))
        return x

    def encode_target(self, m, state, rc, thc, omega, r_in, gamma=1.5, out=None):
        if out is None:
            out = self.torch.empty((self.ncol, self.no), dtype=self.torch.float32,
                                   device=self.device)
        _check(lib().icr_nn_encode_target(self.h, _abi.dptr(m.data_ptr()),
                                          _abi.dptr(state.data_ptr()), _abi.dptr(rc.data_ptr()),
                                          _abi.dptr(thc.data_ptr()), omega, r_in, gamma,
                                          _p(out)))
        return out

    def decode_state(self, m, y, rc, thc, omega, r_in, gamma=1.5):
        st = self.torch.empty((8, self.shape.n_phi, self.shape.n_theta, self.shape.n_r),
                              dtype=self.torch.float64, device=self.device)
        _check(lib().icr_nn_decode_state(self.h, _abi.dptr(m.data_ptr()), _p(y),
                                         _abi.dptr(rc.data_ptr()), _abi.dptr(thc.data_ptr()),
                                         omega, r_in, gamma, _abi.dptr(st.data_ptr())))
        return st


def gemm_bf16(ta, tb, A_bits, B_bits, M, N, K, lda, ldb, bias=None):
    """BF16 product through the library (A_bits, B_bits: torch int16/uint16
    bit patterns on the device) -> torch float32 [M][N]."""
    import torch
    C = torch.empty((M, N), dtype=torch.float32, device=A_bits.device)
    _check(lib().icr_nn_gemm_bf16(ta, tb, M, N, K, _p(A_bits), lda, _p(B_bits), ldb, _p(C), N,
                                  _p(bias) if bias is not None else None,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return C
