"""Python binding of the batched ensemble (icr_ens_* in include/icarus_hip.h).

PyTorch allocates the device workspace; the ensemble's runs are solvers
owned by the library (wrapped as Solver views)."""
from __future__ import annotations

import ctypes

from . import _abi
from ._abi import check, lib
from .solver import Solver, make_grid, make_phys


class Ensemble:
    def __init__(self, grids, *, device=0, stream=None, max_maps=16, max_cmes=4, **phys):
        import torch
        self.grids = list(grids)
        n = len(self.grids)
        self.device = torch.device("cuda", device)
        self.g = (_abi.IcrGrid * n)(*[make_grid(g, max_maps, max_cmes, 0, 2, 0)
                                      for g in self.grids])
        self.p = make_phys(**phys)
        nb = ctypes.c_size_t()
        check(lib().icr_ens_workspace_bytes(n, self.g, ctypes.byref(self.p), ctypes.byref(nb)))
        self.ws_bytes = nb.value
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._ws.data_ptr() + 255) & ~255
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().icr_ens_create(n, self.g, ctypes.byref(self.p), ctypes.c_void_p(ptr),
                                       self.ws_bytes, ctypes.c_void_p(stream.cuda_stream),
                                       ctypes.byref(h)))
        self.h = h
        self.runs = []
        for r in range(n):
            sh = ctypes.c_void_p()
            check(lib().icr_ens_run(self.h, r, ctypes.byref(sh)))
            self.runs.append(Solver.wrap(sh, self.grids[r]))

    def close(self):
        if getattr(self, "h", None):
            for s in self.runs:
                s.h = None
            lib().icr_ens_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_planes(self, r, planes):
        check(lib().icr_ens_set_planes(self.h, r, planes))

    def set_mode(self, persistent=1, grid_blocks=0, use_graphs=1):
        check(lib().icr_ens_set_mode(self.h, int(persistent), int(grid_blocks), int(use_graphs)))

    def step(self, n, t_end=-1.0, raise_on_error=True):
        """Advance every run by up to n steps (stopping at t_end [s] when
        t_end >= 0); per-run records.  With raise_on_error=False a run that
        produced a non-physical cell is reported by its status instead."""
        infos = (_abi.IcrStepInfo * len(self.runs))()
        rc = lib().icr_ens_step(self.h, int(n), float(t_end), infos)
        if raise_on_error or rc != _abi.ICR_ERR_NONPHYSICAL:
            check(rc)
        return [dict(steps=i.steps_taken, status=i.status, t=i.t, dt=i.last_dt,
                     resid=i.residual) for i in infos]
