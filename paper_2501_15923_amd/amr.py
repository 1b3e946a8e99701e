"""Python binding of the block-refined run (icr_amr_* in include/icarus_hip.h).

PyTorch allocates the device workspace; every step of the refined update
runs in the HIP kernels of libicarus_hip.so."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi
from ._abi import check, lib
from .solver import make_grid, make_phys
from .synth import Grid

CRITERIA = {"tracing": 0, "shock": 1, "combined": 2}


class AmrSolver:
    def __init__(self, grid: Grid, *, block=(8, 4, 4), max_level=2, criterion="combined",
                 tau_threshold=0.05, shock_threshold=0.5, regrid_every=5, max_blocks=4096,
                 max_maps=16, max_cmes=4, device=0, stream=None, **phys):
        import torch
        self.grid = grid
        self.bshape = tuple(block)
        self.g = make_grid(grid, max_maps, max_cmes, 0, 2, 0)
        self.p = make_phys(**phys)
        self.q = _abi.IcrAmrParams(block[0], block[1], block[2], max_level, CRITERIA[criterion],
                                   tau_threshold, shock_threshold, regrid_every, max_blocks)
        n = ctypes.c_size_t()
        check(lib().icr_amr_workspace_bytes(ctypes.byref(self.g), ctypes.byref(self.p),
                                            ctypes.byref(self.q), ctypes.byref(n)))
        self.device = torch.device("cuda", device)
        self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._ws.data_ptr() + 255) & ~255
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().icr_amr_create(ctypes.byref(self.g), ctypes.byref(self.p),
                                       ctypes.byref(self.q), ctypes.c_void_p(ptr), n.value,
                                       ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.max_blocks = max_blocks

    def close(self):
        if getattr(self, "h", None):
            lib().icr_amr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_maps(self, times, maps):
        times = np.ascontiguousarray(times, dtype=np.float64)
        maps = np.ascontiguousarray(maps, dtype=np.float64)
        check(lib().icr_amr_set_boundary_maps(self.h, len(times), times.ctypes.data_as(_abi.D),
                                              maps.ctypes.data_as(_abi.D)))

    def set_cmes(self, rows):
        rows = np.ascontiguousarray(np.atleast_2d(rows), dtype=np.float64)
        n = 0 if rows.size == 0 else rows.shape[0]
        check(lib().icr_amr_set_cmes(self.h, n, rows.ctypes.data_as(_abi.D) if n else None))

    def init_radial(self):
        check(lib().icr_amr_init_radial(self.h))

    def step(self, n, t_end=-1.0):
        info = _abi.IcrStepInfo()
        check(lib().icr_amr_step(self.h, int(n), float(t_end), ctypes.byref(info)))
        return dict(steps=info.steps_taken, status=info.status, t=info.t, dt=info.last_dt)

    def force_refine(self, keys):
        k = np.ascontiguousarray(np.asarray(keys, dtype=np.int32).reshape(-1, 4))
        check(lib().icr_amr_force_refine(self.h, len(k),
                                         k.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))

    def leaves(self):
        n = ctypes.c_int()
        keys = np.zeros((self.max_blocks, 4), dtype=np.int32)
        check(lib().icr_amr_leaves(self.h, self.max_blocks,
                                   keys.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                   ctypes.byref(n)))
        return [tuple(r) for r in keys[:n.value].tolist()]

    def n_leaves(self):
        n = ctypes.c_int()
        check(lib().icr_amr_leaves(self.h, 0, None, ctypes.byref(n)))
        return n.value

    def block(self, key):
        br, bt, bp = self.bshape
        out = np.zeros((9, bp, bt, br))
        k = np.ascontiguousarray(np.asarray(key, dtype=np.int32))
        check(lib().icr_amr_get_block(self.h, k.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                      out.ctypes.data_as(_abi.D)))
        return out

    def clock(self):
        c = _abi.IcrClock()
        check(lib().icr_amr_get_clock(self.h, ctypes.byref(c)))
        return dict(t=c.t, step=c.step, last_dt=c.last_dt, next_dt=c.next_dt, t_code=c.t_code)
