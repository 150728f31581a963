"""Thin Python binding of libhemo (C ABI in include/hemo.h).

Argument marshalling only: every step of the coupled update runs in the HIP
kernels of libhemo.so.  PyTorch supplies the device workspace and the
stream.  There is no fallback path: a missing library is an error.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhemo.so")

HC_PERIODIC, HC_WALL = 0, 1
HC_PHI2, HC_PHI4 = 2, 4
KERNELS = ("cell", "lattice", "advect", "interior")
STATUS = {0: "HC_OK", 1: "HC_ERR_ARG", 2: "HC_ERR_STATE", 3: "HC_ERR_DEVICE", 4: "HC_ERR_OOM",
          5: "HC_ERR_NONFINITE", 6: "HC_ERR_UNSUPPORTED"}


class HemoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class LatticeDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("bc", C.c_int32 * 3),
                ("tau", C.c_float), ("body_force", C.c_float * 3), ("wall_u_lo", C.c_float * 3),
                ("wall_u_hi", C.c_float * 3), ("ibm_kernel", C.c_int32),
                ("lees_edwards_u", C.c_float)]


class MeshDesc(C.Structure):
    _fields_ = [("n_vert", C.c_int32), ("n_tri", C.c_int32), ("tri", C.POINTER(C.c_int32)),
                ("rest_pos", C.POINTER(C.c_float))]


_lib = None
_P = C.c_void_p


def _declare(lib):
    i32, i64, sz = C.c_int32, C.c_int64, C.c_size_t
    sig = {
        "hc_create": [_P, _P, i32, _P],
        "hc_set_stream": [_P, _P],
        "hc_query_workspace": [_P, _P],
        "hc_bind_workspace": [_P, _P, sz],
        "hc_set_cells": [_P, i32, _P, _P, _P, _P],
        "hc_init_equilibrium": [_P, C.c_float, _P],
        "hc_step": [_P, i32],
        "hc_sync": [_P],
        "hc_read_populations": [_P, _P, i64],
        "hc_write_populations": [_P, _P, i64],
        "hc_read_macro": [_P, _P, _P, i64],
        "hc_set_field_output": [_P, i32],
        "hc_set_integration": [_P, i32, i32],
        "hc_set_interior_viscosity": [_P, C.c_float],
        "hc_read_interior": [_P, _P, i64],
        "hc_set_cell_viscosity": [_P, _P, i64],
        "hc_read_force_field": [_P, _P, i64],
        "hc_read_vertices": [_P, _P, _P, _P, i64],
        "hc_write_vertices": [_P, _P, _P, i64],
        "hc_read_vertex_velocity": [_P, _P, i64],
        "hc_compute_forces": [_P, _P, _P, i64],
        "hc_read_bins": [_P, _P, _P, _P, i64, _P, _P, i64],
        "hc_num_tiles": [_P, _P],
        "hc_checkpoint_size": [_P, _P],
        "hc_checkpoint_save": [_P, _P, sz],
        "hc_checkpoint_restore": [_P, _P, sz],
        "hc_get_step": [_P, _P],
        "hc_profile": [_P, i32],
        "hc_profile_read": [_P, _P, _P],
        "hc_device_copy": [_P, _P, sz, _P],
        "hc_set_params": [_P, _P, C.c_float],
        "hc_adj_query_workspace": [_P, i32, i32, _P],
        "hc_adj_bind_workspace": [_P, _P, sz, i32, i32],
        "hc_adj_forward": [_P, _P, _P],
        "hc_adj_backward": [_P, _P],
        "hc_adj_multi_forward": [_P, i32, _P, _P],
        "hc_adj_multi_backward": [_P, i32, _P],
        "hc_pack_query_workspace": [_P, i32, _P],
        "hc_pack_run": [_P, _P, _P, _P, i32, i32, _P, sz, _P, _P],
        "hc_pack_run_static": [_P, _P, _P, _P, i32, i32, _P, _P],
        "hc_place_cells": [_P, i32, _P, _P, _P, _P],
        "hc_set_list_capacity": [_P, i32],
        "hc_densest_tile": [_P, _P, _P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.hc_last_error.argtypes = [_P]
    lib.hc_last_error.restype = C.c_char_p
    lib.hc_destroy.argtypes = [_P]
    lib.hc_destroy.restype = None


def load_library(path: str = LIB_PATH):
    """Load libhemo.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} not found: build it with paper_2305_02752_amd/build.py "
                              "(there is no CPU fallback)")
        lib = C.CDLL(path)
        _declare(lib)
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def lattice_desc(lat) -> LatticeDesc:
    d = LatticeDesc()
    d.nx, d.ny, d.nz = int(lat.nx), int(lat.ny), int(lat.nz)
    for i in range(3):
        d.bc[i] = int(lat.bc[i])
        d.body_force[i] = float(lat.body_force[i])
        d.wall_u_lo[i] = float(lat.wall_u_lo[i])
        d.wall_u_hi[i] = float(lat.wall_u_hi[i])
    d.tau = float(lat.tau)
    d.ibm_kernel = int(lat.ibm_kernel)
    d.lees_edwards_u = float(getattr(lat, "lees_edwards_u", 0.0))
    return d


class Simulation:
    """One lattice with up to `max_cells` cells, driven through libhemo.

    lattice: object with nx, ny, nz, bc, tau, body_force, wall_u_lo,
    wall_u_hi, ibm_kernel.  rest_pos float32 [V,3], tri int32 [T,3].
    """

    def __init__(self, lattice, rest_pos, tri, max_cells: int, device: str = "cuda:0",
                 list_capacity: int | None = None):
        """list_capacity: entries per tile list (hc_set_list_capacity), None
        for the library's default."""
        import torch

        self.lib = load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.nx, self.ny, self.nz = int(lattice.nx), int(lattice.ny), int(lattice.nz)
        self.n_sites = self.nx * self.ny * self.nz
        self._rest = np.ascontiguousarray(rest_pos, dtype=np.float32)
        self._tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.nv = self._rest.shape[0]
        self._desc = lattice_desc(lattice)
        mesh = MeshDesc(self.nv, self._tri.shape[0], self._tri.ctypes.data_as(C.POINTER(C.c_int32)),
                        self._rest.ctypes.data_as(C.POINTER(C.c_float)))
        ctx = C.c_void_p()
        rc = self.lib.hc_create(C.byref(self._desc), C.byref(mesh), int(max_cells), C.byref(ctx))
        if rc:
            raise HemoError(rc, self.lib.hc_last_error(None).decode())
        self.ctx = ctx
        self.n_cells = 0
        if list_capacity is not None:
            self._check(self.lib.hc_set_list_capacity(self.ctx, int(list_capacity)))
        nbytes = C.c_size_t()
        self._check(self.lib.hc_query_workspace(self.ctx, C.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        with torch.cuda.device(self.device):
            self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            aligned = (base + 255) & ~255
            self.stream = torch.cuda.current_stream(self.device)
            self._check(self.lib.hc_set_stream(self.ctx, C.c_void_p(self.stream.cuda_stream)))
            self._check(self.lib.hc_bind_workspace(self.ctx, C.c_void_p(aligned), nbytes.value))
        n = C.c_int32()
        self._check(self.lib.hc_num_tiles(self.ctx, C.byref(n)))
        self.n_tiles = n.value

    # ------------------------------------------------------------------ helpers
    def _check(self, rc):
        if rc:
            raise HemoError(rc, self.lib.hc_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.hc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ state
    def set_cells(self, origin, offsets, k, traction=None):
        origin = np.ascontiguousarray(origin, dtype=np.int32)
        offsets = np.ascontiguousarray(offsets, dtype=np.float32)
        k = np.ascontiguousarray(k, dtype=np.float32)
        n = origin.shape[0]
        if offsets.shape != (n, self.nv, 3) or k.shape != (n, 4):
            raise ValueError("cell array shapes")
        tr = None if traction is None else np.ascontiguousarray(traction, dtype=np.float32).reshape(n, 3)
        self._check(self.lib.hc_set_cells(self.ctx, n, _ptr(origin), _ptr(offsets), _ptr(k),
                                          None if tr is None else _ptr(tr)))
        self.n_cells = n

    def init_equilibrium(self, rho0=1.0, u0=(0.0, 0.0, 0.0)):
        u = np.ascontiguousarray(u0, dtype=np.float32)
        self._check(self.lib.hc_init_equilibrium(self.ctx, float(rho0), _ptr(u)))

    def step(self, n: int = 1):
        self._check(self.lib.hc_step(self.ctx, int(n)))

    def sync(self):
        self._check(self.lib.hc_sync(self.ctx))

    def steps_taken(self) -> int:
        s = C.c_int64()
        self._check(self.lib.hc_get_step(self.ctx, C.byref(s)))
        return s.value

    # ------------------------------------------------------------------ read-out
    def read_populations(self) -> np.ndarray:
        out = np.empty((19, self.nz, self.ny, self.nx), dtype=np.float32)
        self._check(self.lib.hc_read_populations(self.ctx, _ptr(out), out.size))
        return out

    def write_populations(self, g):
        g = np.ascontiguousarray(g, dtype=np.float32)
        self._check(self.lib.hc_write_populations(self.ctx, _ptr(g), g.size))

    def set_integration(self, force_every: int = 1, scheme: str = "euler"):
        """Membrane forces every `force_every` steps (held in between) and
        Euler or second-order Adams-Bashforth ("ab2") vertex moves."""
        code = {"euler": 0, "ab2": 1}[scheme]
        self._check(self.lib.hc_set_integration(self.ctx, int(force_every), code))

    def place_cells(self, centres, rot, k, traction=None):
        """Cells from packed ellipsoids on the device: centres [n,3] and rot
        [n,3,3] (or [n,9]) float32 device tensors; k [n,4] and traction
        [n,3] host arrays."""
        n = int(centres.shape[0])
        kk = np.ascontiguousarray(k, dtype=np.float32).reshape(n, 4)
        tr = None if traction is None else np.ascontiguousarray(traction, dtype=np.float32).reshape(n, 3)
        self._check(self.lib.hc_place_cells(self.ctx, n, C.c_void_p(centres.data_ptr()),
                                            C.c_void_p(rot.data_ptr()), _ptr(kk),
                                            None if tr is None else _ptr(tr)))
        self.n_cells = n

    def set_interior_viscosity(self, ratio: float):
        """Sites inside the cells relax with `ratio` times the plasma
        viscosity (1: off)."""
        self._check(self.lib.hc_set_interior_viscosity(self.ctx, float(ratio)))

    def set_cell_viscosity(self, ratio):
        """One interior viscosity ratio per cell (at most 8 distinct)."""
        r = np.ascontiguousarray(ratio, dtype=np.float32).reshape(-1)
        self._check(self.lib.hc_set_cell_viscosity(self.ctx, _ptr(r), r.size))

    def read_interior(self):
        """Inside marks of the current positions, uint8 [nz, ny, nx]: 1 << k
        inside a cell of viscosity class k (distinct ratios in increasing
        order; the highest class where cells overlap), 0 outside."""
        m = np.empty((self.nz, self.ny, self.nx), dtype=np.uint8)
        self._check(self.lib.hc_read_interior(self.ctx, _ptr(m), m.size))
        return m

    def set_field_output(self, enable: bool):
        """Whether each step writes its force and (u, rho) fields out (for
        read_force_field / read_macro); the step itself keeps them on chip."""
        self._check(self.lib.hc_set_field_output(self.ctx, 1 if enable else 0))

    def read_macro(self):
        rho = np.empty((self.nz, self.ny, self.nx), dtype=np.float32)
        u = np.empty((3, self.nz, self.ny, self.nx), dtype=np.float32)
        self._check(self.lib.hc_read_macro(self.ctx, _ptr(rho), _ptr(u), self.n_sites))
        return rho, u

    def read_force_field(self):
        f = np.empty((3, self.nz, self.ny, self.nx), dtype=np.float32)
        self._check(self.lib.hc_read_force_field(self.ctx, _ptr(f), self.n_sites))
        return f

    def read_vertices(self):
        o = np.empty((self.n_cells, 3), dtype=np.int32)
        off = np.empty((self.n_cells, self.nv, 3), dtype=np.float32)
        fv = np.empty((self.n_cells, self.nv, 3), dtype=np.float32)
        self._check(self.lib.hc_read_vertices(self.ctx, _ptr(o), _ptr(off), _ptr(fv), self.n_cells))
        return o, off, fv

    def read_vertex_velocity(self):
        vel = np.empty((self.n_cells, self.nv, 3), dtype=np.float32)
        self._check(self.lib.hc_read_vertex_velocity(self.ctx, _ptr(vel), self.n_cells))
        return vel

    def write_vertices(self, origin, offsets):
        origin = np.ascontiguousarray(origin, dtype=np.int32)
        offsets = np.ascontiguousarray(offsets, dtype=np.float32)
        self._check(self.lib.hc_write_vertices(self.ctx, _ptr(origin), _ptr(offsets), self.n_cells))

    def densest_tile(self):
        """(entries of the fullest tile list for the current positions, capacity)."""
        e, cap = C.c_int32(), C.c_int32()
        self._check(self.lib.hc_densest_tile(self.ctx, C.byref(e), C.byref(cap)))
        return e.value, cap.value

    def compute_forces(self):
        a = np.empty(self.n_cells, dtype=np.float64)
        v = np.empty(self.n_cells, dtype=np.float64)
        self._check(self.lib.hc_compute_forces(self.ctx, _ptr(a), _ptr(v), self.n_cells))
        _, _, fv = self.read_vertices()
        return fv, a, v

    def read_bins(self):
        nt = self.n_tiles
        owner = np.empty(self.n_cells * self.nv, dtype=np.int32)
        tptr = np.empty(nt + 1, dtype=np.int32)
        cptr = np.empty(nt + 1, dtype=np.int32)
        cap_t = self.n_cells * self.nv * 27
        cap_c = self.n_cells * 512   # a cell covers at most 8 tiles per axis in the read-out
        touch = np.empty(max(cap_t, 1), dtype=np.int32)
        cells = np.empty(max(cap_c, 1), dtype=np.int32)
        self._check(self.lib.hc_read_bins(self.ctx, _ptr(owner), _ptr(tptr), _ptr(touch), touch.size,
                                          _ptr(cptr), _ptr(cells), cells.size))
        return owner, tptr, touch[:tptr[-1]].copy(), cptr, cells[:cptr[-1]].copy()

    def profile(self, enable: bool = True):
        self._check(self.lib.hc_profile(self.ctx, int(enable)))

    def profile_read(self) -> dict:
        ms = np.zeros(len(KERNELS), dtype=np.float64)
        n = np.zeros(len(KERNELS), dtype=np.int64)
        self._check(self.lib.hc_profile_read(self.ctx, _ptr(ms), _ptr(n)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNELS)}

    def set_params(self, k=None, tau=None):
        """Replace per-cell stiffnesses k [C,4] and/or the relaxation time."""
        kk = None if k is None else np.ascontiguousarray(k, dtype=np.float32).reshape(self.n_cells, 4)
        t = float(self._desc.tau if tau is None else tau)
        self._check(self.lib.hc_set_params(self.ctx, None if kk is None else _ptr(kk), t))
        self._desc.tau = t

    def adj_bind(self, n_steps: int, ckpt_every: int):
        """Allocate and bind the reverse-mode workspace for runs of n_steps."""
        nb = C.c_size_t()
        self._check(self.lib.hc_adj_query_workspace(self.ctx, int(n_steps), int(ckpt_every), C.byref(nb)))
        with self.torch.cuda.device(self.device):
            self._adj_ws = self.torch.empty(nb.value + 256, dtype=self.torch.uint8, device=self.device)
        aligned = (self._adj_ws.data_ptr() + 255) & ~255
        self._check(self.lib.hc_adj_bind_workspace(self.ctx, C.c_void_p(aligned), nb.value, int(n_steps),
                                                   int(ckpt_every)))
        self.adj_workspace_bytes = nb.value

    def adj_forward(self, targets) -> np.ndarray:
        t = np.ascontiguousarray(targets, dtype=np.float64).reshape(self.n_cells, 2)
        loss = np.empty(self.n_cells, dtype=np.float64)
        self._check(self.lib.hc_adj_forward(self.ctx, _ptr(t), _ptr(loss)))
        return loss

    def adj_backward(self) -> np.ndarray:
        g = np.empty((self.n_cells, 5), dtype=np.float64)
        self._check(self.lib.hc_adj_backward(self.ctx, _ptr(g)))
        return g

    @staticmethod
    def _ctx_array(sims):
        arr = (C.c_void_p * len(sims))(*[s.ctx for s in sims])
        return arr

    @staticmethod
    def adj_multi_forward(sims, targets) -> np.ndarray:
        """hc_adj_multi_forward over boxes of one shape: every per-step kernel
        is one launch over all boxes (on the first box's stream).  targets
        [B][cells][2]; returns the losses [B][cells]."""
        n, nc = len(sims), sims[0].n_cells
        t = np.ascontiguousarray(targets, dtype=np.float64).reshape(n, nc, 2)
        loss = np.empty((n, nc), dtype=np.float64)
        arr = Simulation._ctx_array(sims)
        sims[0]._check(sims[0].lib.hc_adj_multi_forward(C.cast(arr, C.c_void_p), n, _ptr(t), _ptr(loss)))
        return loss

    @staticmethod
    def adj_multi_backward(sims) -> np.ndarray:
        """hc_adj_multi_backward: gradients [B][cells][5] of the last
        hc_adj_multi_forward."""
        n, nc = len(sims), sims[0].n_cells
        g = np.empty((n, nc, 5), dtype=np.float64)
        arr = Simulation._ctx_array(sims)
        sims[0]._check(sims[0].lib.hc_adj_multi_backward(C.cast(arr, C.c_void_p), n, _ptr(g)))
        return g

    def checkpoint_save(self) -> bytes:
        n = C.c_size_t()
        self._check(self.lib.hc_checkpoint_size(self.ctx, C.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        self._check(self.lib.hc_checkpoint_save(self.ctx, _ptr(buf), buf.size))
        return buf

    def checkpoint_restore(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.lib.hc_checkpoint_restore(self.ctx, _ptr(buf), buf.size))


def device_copy(dst, src, nbytes: int, stream_handle: int):
    """Library streaming copy (bandwidth reference) between two device buffers."""
    lib = load_library()
    rc = lib.hc_device_copy(C.c_void_p(dst), C.c_void_p(src), int(nbytes), C.c_void_p(stream_handle))
    if rc:
        raise HemoError(rc, lib.hc_last_error(None).decode())


class PackDesc(C.Structure):
    _fields_ = [("box", C.c_float * 3), ("periodic", C.c_int32 * 3), ("lo", C.c_float * 3),
                ("hi", C.c_float * 3), ("max_semi", C.c_float), ("eta", C.c_float),
                ("max_move", C.c_float), ("quad", C.c_int32)]


class Packer:
    """Force-bias packing of surrogate ellipsoids on the device.

    box, periodic: domain sides and per-axis periodicity; lo, hi: allowed
    extent on wall axes; max_semi: bound on every semi-axis; eta: move per
    unit overlapping volume; max_move: longest move per iteration; quad:
    quadrature grid per axis (4, 8 or 16).
    """

    def __init__(self, box, periodic, lo=(0.0, 0.0, 0.0), hi=(0.0, 0.0, 0.0), max_semi=9.0,
                 eta=0.03, max_move=1.0, quad=8, device: str = "cuda:0"):
        import torch
        self.lib = load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.desc = PackDesc((C.c_float * 3)(*box), (C.c_int32 * 3)(*[1 if p else 0 for p in periodic]),
                             (C.c_float * 3)(*lo), (C.c_float * 3)(*hi), float(max_semi), float(eta),
                             float(max_move), int(quad))
        self._ws = None

    def _check(self, rc):
        if rc:
            raise HemoError(rc, self.lib.hc_last_error(None).decode())

    def workspace(self, n: int):
        nbytes = C.c_size_t()
        self._check(self.lib.hc_pack_query_workspace(C.byref(self.desc), int(n), C.byref(nbytes)))
        if self._ws is None or self._ws.numel() < nbytes.value + 256:
            self._ws = self.torch.empty(nbytes.value + 256, dtype=self.torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        return (base + 255) & ~255, nbytes.value

    def run_device(self, centres, rot, semi, n_iter: int, measure: bool = True):
        """Iterate on device tensors (float32, contiguous): centres [n,3]
        in place, rot [n,3,3], semi [n,3].  Returns the overlap record
        (initial volume, pairs, final volume, pairs) or None."""
        n = int(centres.shape[0])
        ws, nbytes = self.workspace(n)
        out = np.zeros(4, dtype=np.float64)
        stream = self.torch.cuda.current_stream(self.device).cuda_stream
        self._check(self.lib.hc_pack_run(C.byref(self.desc), C.c_void_p(centres.data_ptr()),
                                         C.c_void_p(rot.data_ptr()), C.c_void_p(semi.data_ptr()), n,
                                         int(n_iter), C.c_void_p(ws), nbytes, C.c_void_p(stream),
                                         _ptr(out) if measure else None))
        return tuple(out) if measure else None

    def run_device_static(self, centres, rot, semi, n_iter: int, measure: bool = True):
        """As run_device, through hc_pack_run_static: the library's static
        per-device scratch instead of a workspace (nothing allocated)."""
        n = int(centres.shape[0])
        out = np.zeros(4, dtype=np.float64)
        stream = self.torch.cuda.current_stream(self.device).cuda_stream
        self._check(self.lib.hc_pack_run_static(C.byref(self.desc), C.c_void_p(centres.data_ptr()),
                                                C.c_void_p(rot.data_ptr()), C.c_void_p(semi.data_ptr()), n,
                                                int(n_iter), C.c_void_p(stream), _ptr(out) if measure else None))
        return tuple(out) if measure else None

    def run(self, centres, rot, semi, n_iter: int):
        """Host arrays in, (centres [n,3] float32, overlap record) out."""
        t = self.torch
        c = t.tensor(np.ascontiguousarray(centres, dtype=np.float32), device=self.device)
        r = t.tensor(np.ascontiguousarray(rot, dtype=np.float32).reshape(-1, 9), device=self.device)
        s = t.tensor(np.ascontiguousarray(semi, dtype=np.float32), device=self.device)
        rec = self.run_device(c, r, s, n_iter)
        return c.cpu().numpy(), rec


def _declare_batch(lib):
    i32, i64, sz = C.c_int32, C.c_int64, C.c_size_t
    sig = {
        "hc_batch_create": [i32, _P, _P, _P],
        "hc_batch_set_stream": [_P, _P],
        "hc_batch_query_workspace": [_P, _P],
        "hc_batch_bind_workspace": [_P, _P, sz],
        "hc_batch_set_cells": [_P, _P, _P, _P, _P],
        "hc_batch_set_tiling": [_P, i32, i32, i32],
        "hc_batch_set_interior_viscosity": [_P, _P],
        "hc_batch_get_tiling": [_P, _P, _P, _P, _P],
        "hc_batch_autotune": [_P, C.c_char_p, i32, _P, _P, _P],
        "hc_batch_run": [_P, i32],
        "hc_batch_sync": [_P],
        "hc_batch_box_steps": [_P, i32, _P],
        "hc_batch_read_populations": [_P, i32, _P, i64],
        "hc_batch_write_populations": [_P, i32, _P, i64],
        "hc_batch_read_vertices": [_P, i32, _P, _P, _P, _P],
        "hc_batch_launches": [_P, _P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.hc_batch_last_error.argtypes = [_P]
    lib.hc_batch_last_error.restype = C.c_char_p
    lib.hc_batch_destroy.argtypes = [_P]
    lib.hc_batch_destroy.restype = None


class Batch:
    """Independent single-cell boxes advanced by one persistent launch per run."""

    def __init__(self, lattices, rest_pos, tri, device: str = "cuda:0"):
        import torch

        self.lib = load_library()
        if not hasattr(self.lib, "_batch_declared"):
            _declare_batch(self.lib)
            self.lib._batch_declared = True
        self.device = torch.device(device)
        self.lats = list(lattices)
        self.n_boxes = len(self.lats)
        self._rest = np.ascontiguousarray(rest_pos, dtype=np.float32)
        self._tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.nv = self._rest.shape[0]
        descs = (LatticeDesc * self.n_boxes)(*[lattice_desc(l) for l in self.lats])
        self._descs = descs
        mesh = MeshDesc(self.nv, self._tri.shape[0], self._tri.ctypes.data_as(C.POINTER(C.c_int32)),
                        self._rest.ctypes.data_as(C.POINTER(C.c_float)))
        h = C.c_void_p()
        rc = self.lib.hc_batch_create(self.n_boxes, C.cast(descs, C.c_void_p), C.byref(mesh), C.byref(h))
        if rc:
            raise HemoError(rc, self.lib.hc_batch_last_error(None).decode())
        self.h = h
        nbytes = C.c_size_t()
        self._check(self.lib.hc_batch_query_workspace(self.h, C.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        with torch.cuda.device(self.device):
            self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
            aligned = (self._ws.data_ptr() + 255) & ~255
            self.stream = torch.cuda.current_stream(self.device)
            self._check(self.lib.hc_batch_set_stream(self.h, C.c_void_p(self.stream.cuda_stream)))
            self._check(self.lib.hc_batch_bind_workspace(self.h, C.c_void_p(aligned), nbytes.value))

    def _check(self, rc):
        if rc:
            raise HemoError(rc, self.lib.hc_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.hc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_cells(self, origin, offsets, k, traction=None):
        origin = np.ascontiguousarray(origin, dtype=np.int32).reshape(self.n_boxes, 3)
        offsets = np.ascontiguousarray(offsets, dtype=np.float32).reshape(self.n_boxes, self.nv, 3)
        k = np.ascontiguousarray(k, dtype=np.float32).reshape(self.n_boxes, 4)
        tr = None if traction is None else np.ascontiguousarray(traction, dtype=np.float32).reshape(self.n_boxes, 3)
        self._check(self.lib.hc_batch_set_cells(self.h, _ptr(origin), _ptr(offsets), _ptr(k),
                                                None if tr is None else _ptr(tr)))

    def set_interior_viscosity(self, ratios):
        """Viscosity ratio inside each box's cell (one float per box)."""
        r = np.ascontiguousarray(np.broadcast_to(np.asarray(ratios, dtype=np.float32), (self.n_boxes,)))
        self._check(self.lib.hc_batch_set_interior_viscosity(self.h, _ptr(r)))

    def set_tiling(self, ty, tz, block=256):
        self._check(self.lib.hc_batch_set_tiling(self.h, int(ty), int(tz), int(block)))

    def tiling(self):
        v = [C.c_int32() for _ in range(4)]
        self._check(self.lib.hc_batch_get_tiling(self.h, *[C.byref(x) for x in v]))
        return {"ty": v[0].value, "tz": v[1].value, "block": v[2].value, "grid": v[3].value}

    def autotune(self, cache_path=None, trial_steps=10):
        v = [C.c_int32() for _ in range(3)]
        path = None if cache_path is None else str(cache_path).encode()
        self._check(self.lib.hc_batch_autotune(self.h, path, int(trial_steps), *[C.byref(x) for x in v]))
        return {"ty": v[0].value, "tz": v[1].value, "block": v[2].value}

    def run(self, n):
        self._check(self.lib.hc_batch_run(self.h, int(n)))

    def sync(self):
        self._check(self.lib.hc_batch_sync(self.h))

    def box_steps(self, box):
        s = C.c_int64()
        self._check(self.lib.hc_batch_box_steps(self.h, int(box), C.byref(s)))
        return s.value

    def launches(self):
        s = C.c_int64()
        self._check(self.lib.hc_batch_launches(self.h, C.byref(s)))
        return s.value

    def _shape(self, box):
        l = self.lats[box]
        return (19, l.nz, l.ny, l.nx)

    def read_populations(self, box):
        out = np.empty(self._shape(box), dtype=np.float32)
        self._check(self.lib.hc_batch_read_populations(self.h, int(box), _ptr(out), out.size))
        return out

    def write_populations(self, box, g):
        g = np.ascontiguousarray(g, dtype=np.float32)
        self._check(self.lib.hc_batch_write_populations(self.h, int(box), _ptr(g), g.size))

    def read_vertices(self, box):
        o = np.empty(3, dtype=np.int32)
        off = np.empty((self.nv, 3), dtype=np.float32)
        f = np.empty((self.nv, 3), dtype=np.float32)
        vel = np.empty((self.nv, 3), dtype=np.float32)
        self._check(self.lib.hc_batch_read_vertices(self.h, int(box), _ptr(o), _ptr(off), _ptr(f), _ptr(vel)))
        return o, off, f, vel
