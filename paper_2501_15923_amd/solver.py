"""Thin Python binding over the C-ABI (include/icarus_hip.h).

PyTorch provides the device workspace and the stream; every step of the
update runs in the HIP kernels of libicarus_hip.so.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi
from ._abi import check, lib
from .synth import AU, DEG, Grid, OMEGA_SUN


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(_abi.D)


def make_grid(grid: Grid, max_maps=16, max_cmes=4, max_probes=8, max_traj_pts=1024,
              probe_log_rows=0):
    return _abi.IcrGrid(grid.nr, grid.nt, grid.np_, grid.r_in, grid.r_out, grid.th_min,
                        grid.th_max, max_maps, max_cmes, max_probes, max_traj_pts,
                        probe_log_rows)


def make_phys(gamma=1.5, omega=OMEGA_SUN, cfl=0.4, flux=_abi.FLUX_TVDLF,
              limiter=_abi.LIM_MINMOD, precision=64, gravity=True, corotation=True,
              tracer=False, bc_transverse=_abi.BCT_MAP):
    return _abi.IcrPhys(gamma, omega, cfl, flux, limiter, precision, int(gravity),
                        int(corotation), int(tracer), int(bc_transverse))


class Solver:
    def __init__(self, grid: Grid, *, gamma=1.5, omega=OMEGA_SUN, cfl=0.4,
                 flux=_abi.FLUX_TVDLF, limiter=_abi.LIM_MINMOD, precision=64,
                 gravity=True, corotation=True, tracer=False, bc_transverse=_abi.BCT_MAP,
                 max_maps=16, max_cmes=4, max_probes=8,
                 max_traj_pts=1024, probe_log_rows=0, device=0, stream=None):
        import torch
        self.torch = torch
        self.grid = grid
        self.owned = True
        self.device = torch.device("cuda", device)
        self.g = make_grid(grid, max_maps, max_cmes, max_probes, max_traj_pts, probe_log_rows)
        self.p = make_phys(gamma, omega, cfl, flux, limiter, precision, gravity, corotation,
                           tracer, bc_transverse)
        self.probe_log_rows = probe_log_rows
        nbytes = ctypes.c_size_t()
        check(lib().icr_workspace_bytes(ctypes.byref(self.g), ctypes.byref(self.p),
                                        ctypes.byref(nbytes)))
        self.ws_bytes = nbytes.value
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().icr_create(ctypes.byref(self.g), ctypes.byref(self.p),
                                   ctypes.c_void_p(self.ws_ptr), self.ws_bytes,
                                   ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.n_probes = 0

    @classmethod
    def wrap(cls, handle, grid: Grid, probe_log_rows=0):
        """A view of a solver owned elsewhere (an ensemble run)."""
        self = cls.__new__(cls)
        self.grid = grid
        self.owned = False
        self.h = handle
        self.n_probes = 0
        self.probe_log_rows = probe_log_rows
        return self

    def _device_tensor(self, a, shape, what):
        """Check a torch tensor handed to the library by pointer: float64,
        contiguous, the expected element count, on a GPU."""
        import torch
        if a.dtype != torch.float64:
            raise TypeError(f"{what} must be float64 (got {a.dtype})")
        if not a.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        if a.numel() != int(np.prod(shape)):
            raise ValueError(f"{what} must have {int(np.prod(shape))} elements {shape} "
                             f"(got {a.numel()})")
        if a.device.type != "cuda":
            raise ValueError(f"{what} must be on the GPU (got {a.device})")
        return _abi.dptr(a.data_ptr())

    def close(self):
        if getattr(self, "h", None):
            if self.owned:
                lib().icr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (8, self.grid.np_, self.grid.nt, self.grid.nr)

    # ---- setup -----------------------------------------------------------
    def edges(self):
        r = np.zeros(self.grid.nr + 1)
        t = np.zeros(self.grid.nt + 1)
        p = np.zeros(self.grid.np_ + 1)
        check(lib().icr_grid_edges(self.h, _np_ptr(r), _np_ptr(t), _np_ptr(p)))
        return r, t, p

    def set_maps(self, times, maps):
        times = np.ascontiguousarray(times, dtype=np.float64)
        maps = np.ascontiguousarray(maps, dtype=np.float64)
        check(lib().icr_set_boundary_maps(self.h, len(times), _np_ptr(times), _np_ptr(maps), 0))

    def append_maps(self, times, maps):
        """Stream later maps in (older ones the clock has passed are dropped);
        returns the number of maps held."""
        times = np.ascontiguousarray(np.atleast_1d(times), dtype=np.float64)
        maps = np.ascontiguousarray(maps, dtype=np.float64).reshape(
            (len(times), 8, self.grid.nt, self.grid.np_))
        held = ctypes.c_int()
        check(lib().icr_append_boundary_maps(self.h, len(times), _np_ptr(times), _np_ptr(maps),
                                             0, ctypes.byref(held)))
        return held.value

    def set_cmes(self, rows):
        rows = np.ascontiguousarray(np.atleast_2d(rows), dtype=np.float64)
        n = 0 if rows.size == 0 else rows.shape[0]
        check(lib().icr_set_cmes(self.h, n, _np_ptr(rows) if n else None))

    def init_radial(self):
        check(lib().icr_init_radial(self.h))

    def set_state(self, a, kind=_abi.STATE_PRIM_SI):
        if hasattr(a, "data_ptr"):
            check(lib().icr_set_state(self.h, self._device_tensor(a, self.shape, "state"),
                                      kind, 1))
        else:
            a = np.ascontiguousarray(a, dtype=np.float64)
            check(lib().icr_set_state(self.h, _np_ptr(a), kind, 0))

    def get_state(self, kind=_abi.STATE_PRIM_SI):
        out = np.zeros(self.shape)
        check(lib().icr_get_state(self.h, _np_ptr(out), kind, 0))
        return out

    def get_state_device(self, kind=_abi.STATE_PRIM_SI):
        """The state as a torch float64 tensor on the device."""
        import torch
        out = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        check(lib().icr_get_state(self.h, _abi.dptr(out.data_ptr()), kind, 1))
        return out

    def clock(self):
        c = _abi.IcrClock()
        check(lib().icr_get_clock(self.h, ctypes.byref(c)))
        return dict(t=c.t, step=c.step, last_dt=c.last_dt, next_dt=c.next_dt,
                    resid=c.residual, t_code=c.t_code)

    def set_clock(self, t, step=0):
        check(lib().icr_set_clock(self.h, float(t), int(step)))

    def set_clock_code(self, t_code, step=0):
        check(lib().icr_set_clock_code(self.h, float(t_code), int(step)))

    def step(self, n, t_end=-1.0, raise_on_error=True):
        info = _abi.IcrStepInfo()
        rc = lib().icr_step(self.h, int(n), float(t_end), ctypes.byref(info))
        if raise_on_error:
            check(rc)
        return dict(rc=rc, steps=info.steps_taken, status=info.status, bad_cell=info.bad_cell,
                    t=info.t, dt=info.last_dt, resid=info.residual)

    def set_probes(self, traj, cadence=-1.0):
        traj = np.ascontiguousarray(traj, dtype=np.float64)
        self.n_probes = traj.shape[0]
        check(lib().icr_set_probes(self.h, traj.shape[0], traj.shape[1], _np_ptr(traj),
                                   float(cadence)))

    def sample_probes(self):
        out = np.zeros((self.n_probes, 12))
        check(lib().icr_sample_probes(self.h, _np_ptr(out)))
        return out

    def read_probe_log(self, cap=100000):
        """(records [n][n_probes][12], number logged).  The device log keeps
        the first probe_log_rows records; logging more raises instead of
        returning a silently truncated series."""
        out = np.zeros((cap, self.n_probes, 12))
        n = ctypes.c_int()
        check(lib().icr_read_probe_log(self.h, _np_ptr(out), cap, ctypes.byref(n)))
        if n.value > self.probe_log_rows:
            raise RuntimeError(f"probe log overflow: {n.value} records logged, the device log "
                               f"holds {self.probe_log_rows} (raise probe_log_rows)")
        return out[:min(n.value, cap, self.probe_log_rows)], n.value

    def set_tracer(self, tau):
        """CME mass fraction tau [n_phi][n_theta][n_r] (scalar broadcasts)."""
        if hasattr(tau, "data_ptr"):
            check(lib().icr_set_tracer(self.h, self._device_tensor(tau, self.shape[1:], "tau"), 1))
            return
        tau = np.ascontiguousarray(np.broadcast_to(tau, self.shape[1:]), dtype=np.float64)
        check(lib().icr_set_tracer(self.h, _np_ptr(tau), 0))

    def get_tracer(self):
        out = np.zeros(self.shape[1:])
        check(lib().icr_get_tracer(self.h, _np_ptr(out), 0))
        return out

    def divv(self):
        """Velocity divergence [1/s], [n_phi][n_theta][n_r]."""
        out = np.zeros(self.shape[1:])
        check(lib().icr_divv(self.h, _np_ptr(out), 0))
        return out

    def shell(self, r):
        """rho and v_r on the sphere of radius r [m]: [2][n_theta][n_phi]."""
        out = np.zeros((2, self.grid.nt, self.grid.np_))
        check(lib().icr_sample_shell(self.h, float(r), _np_ptr(out)))
        return out

    def boundary_at(self, t):
        out = np.zeros((8, self.grid.nt, self.grid.np_))
        check(lib().icr_boundary_at(self.h, float(t), _np_ptr(out)))
        return out

    def set_launch(self, variant=0, tile_r=0, tile_t=0, use_graphs=1):
        check(lib().icr_set_launch(self.h, variant, tile_r, tile_t, use_graphs))

    def profile_steps(self, n):
        """Mean ms per launch of (boundary, stage 1, stage 2, probe logger)."""
        out = np.zeros(4)
        check(lib().icr_profile_steps(self.h, int(n), _np_ptr(out)))
        return out


def units() -> dict:
    out = np.zeros(6)
    check(lib().icr_units(_np_ptr(out)))
    return dict(t=out[0], L=out[1], rho=out[2], p=out[3], B=out[4], v=out[5])
