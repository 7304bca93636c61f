"""ctypes binding of libcpm (include/cpm.h) with torch tensors as device memory.

Only argument marshalling happens here: every step of the path runs in the
HIP kernels of libcpm.so.  torch is imported before the library is loaded so
that the process uses one HIP runtime (torch's) for both.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpm.so")

CPM_OK, CPM_EINVAL, CPM_ESTATE, CPM_ENOTSPD, CPM_EDEVICE, CPM_ENOMEM, CPM_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
FINITE_FIELD, DOUBLED_CELL, SLAB = 0, 1, 2
GEOMETRY = {"ff": FINITE_FIELD, "dc": DOUBLED_CELL, "slab": SLAB}
KSPACE_EWALD, KSPACE_PPPM = 0, 1
FP64, MIXED = 0, 1
FLAG_GRAPH = 1
(BUF_CELL_START, BUF_SITE_ORDER, BUF_PHI_REAL, BUF_B, BUF_RHO_MESH, BUF_PHI_MESH, BUF_FIELD_MESH, BUF_NCELL,
 BUF_BATCH_CHUNK) = range(9)
KERNELS = ("bin", "real_b", "site_pairs", "fft_xy_fwd", "fft_z_pot", "fft_xy_inv", "gather_b", "charges",
           "spread_elec", "fft_xy_fwd_e", "fft_z_field", "fft_xy_inv_e", "site_forces", "energy",
           "gemm", "expand_q", "expand_f")

_STATUS_NAMES = {0: "CPM_OK", -1: "CPM_EINVAL", -2: "CPM_ESTATE", -3: "CPM_ENOTSPD", -4: "CPM_EDEVICE",
                 -5: "CPM_ENOMEM", -6: "CPM_ENONFINITE"}

EXPORTED = ("cpm_create", "cpm_set_stream", "cpm_build_elastance", "cpm_solve", "cpm_solve_batch",
            "cpm_grad", "cpm_get_matrix", "cpm_set_matrix", "cpm_get_buffer", "cpm_sync_status",
            "cpm_last_error", "cpm_destroy", "cpm_replay_kernel", "cpm_profile", "cpm_profile_noalloc",
            "cpm_md_create", "cpm_md_run", "cpm_md_state", "cpm_md_set_thermostat", "cpm_md_destroy",
            "cpm_set_batch_shape")


class MDDesc(ctypes.Structure):
    _fields_ = [
        ("n_mol", ctypes.c_int),
        ("mol_size", ctypes.POINTER(ctypes.c_int)),
        ("mol_group", ctypes.POINTER(ctypes.c_int)),
        ("n_groups", ctypes.c_int),
        ("site_mass", ctypes.POINTER(ctypes.c_double)),
        ("site_sigma", ctypes.POINTER(ctypes.c_double)),
        ("site_eps", ctypes.POINTER(ctypes.c_double)),
        ("n_lj_elec", ctypes.c_int),
        ("lj_elec_xyz", ctypes.POINTER(ctypes.c_double)),
        ("carbon_sigma", ctypes.c_double), ("carbon_eps", ctypes.c_double),
        ("lj_cut", ctypes.c_double), ("bond", ctypes.c_double), ("dt", ctypes.c_double),
        ("temperature", ctypes.c_double), ("tau", ctypes.c_double),
        ("charge_every", ctypes.c_int),
    ]


class CpmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class CpmDesc(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double * 3),
        ("geometry", ctypes.c_int), ("kspace", ctypes.c_int), ("precision", ctypes.c_int),
        ("eta", ctypes.c_double), ("alpha", ctypes.c_double), ("rcut", ctypes.c_double), ("kcut", ctypes.c_double),
        ("mesh", ctypes.c_int * 3), ("order", ctypes.c_int),
        ("alpha_build", ctypes.c_double), ("rcut_build", ctypes.c_double), ("kcut_build", ctypes.c_double),
        ("n_elec", ctypes.c_int),
        ("elec_xyz", ctypes.POINTER(ctypes.c_double)),
        ("elec_side", ctypes.POINTER(ctypes.c_int8)),
        ("elec_sub", ctypes.POINTER(ctypes.c_uint8)),
        ("n_site", ctypes.c_int),
        ("site_q", ctypes.POINTER(ctypes.c_double)),
        ("flags", ctypes.c_int),
    ]


_lib = None


def load_library():
    """Load libcpm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2201_12963_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    lib.cpm_create.argtypes = [ctypes.POINTER(CpmDesc), vp, ctypes.POINTER(vp)]
    lib.cpm_create.restype = ip
    lib.cpm_set_stream.argtypes = [vp, vp]
    lib.cpm_set_stream.restype = ip
    lib.cpm_build_elastance.argtypes = [vp]
    lib.cpm_build_elastance.restype = ip
    lib.cpm_solve.argtypes = [vp, vp, ctypes.c_double, vp, vp, vp]
    lib.cpm_solve.restype = ip
    lib.cpm_solve_batch.argtypes = [vp, ip, vp, ip, dp, vp, vp, vp]
    lib.cpm_solve_batch.restype = ip
    lib.cpm_grad.argtypes = [vp, vp, ctypes.c_double, vp, vp, vp, vp, vp]
    lib.cpm_grad.restype = ip
    lib.cpm_get_matrix.argtypes = [vp, ip, dp]
    lib.cpm_get_matrix.restype = ip
    lib.cpm_set_matrix.argtypes = [vp, dp]
    lib.cpm_set_matrix.restype = ip
    lib.cpm_get_buffer.argtypes = [vp, ip, vp]
    lib.cpm_get_buffer.restype = ctypes.c_longlong
    lib.cpm_profile.argtypes = [vp, ip, vp, vp, ctypes.c_longlong, ctypes.c_double, ip, ctypes.c_double,
                                ctypes.c_double, vp, vp]
    lib.cpm_profile.restype = ip
    lib.cpm_profile_noalloc.argtypes = lib.cpm_profile.argtypes
    lib.cpm_profile_noalloc.restype = ip
    lib.cpm_md_create.argtypes = [vp, ctypes.POINTER(MDDesc), ctypes.POINTER(vp)]
    lib.cpm_md_create.restype = ip
    lib.cpm_md_run.argtypes = [vp, vp, vp, ctypes.c_double, ip, vp, vp]
    lib.cpm_md_run.restype = ip
    lib.cpm_md_state.argtypes = [vp, dp, dp, ctypes.POINTER(ctypes.c_longlong)]
    lib.cpm_md_state.restype = ip
    lib.cpm_md_set_thermostat.argtypes = [vp, ip]
    lib.cpm_md_set_thermostat.restype = ip
    lib.cpm_md_destroy.argtypes = [vp]
    lib.cpm_md_destroy.restype = None
    lib.cpm_set_batch_shape.argtypes = [vp, ip, ip, ip]
    lib.cpm_set_batch_shape.restype = ip
    lib.cpm_replay_kernel.argtypes = [vp, ip, ip]
    lib.cpm_replay_kernel.restype = ip
    lib.cpm_sync_status.argtypes = [vp]
    lib.cpm_sync_status.restype = ip
    lib.cpm_last_error.argtypes = [vp]
    lib.cpm_last_error.restype = ctypes.c_char_p
    lib.cpm_destroy.argtypes = [vp]
    lib.cpm_destroy.restype = None
    _lib = lib
    return lib


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float64:
        raise ValueError("device arguments must be contiguous float64 tensors on the GPU")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One electrode geometry plus its per-step buffers (wraps cpm_ctx)."""

    def __init__(self, *, box, geometry, kspace, precision, eta, alpha, rcut, kcut, mesh, order,
                 alpha_build, rcut_build, kcut_build, elec_xyz, elec_side, elec_sub, site_q,
                 stream: Optional[torch.cuda.Stream] = None, graph: bool = False):
        self._lib = load_library()
        self._ctx = ctypes.c_void_p()
        self._keep = []
        d = CpmDesc()
        d.box[:] = [float(b) for b in box]
        d.geometry, d.kspace, d.precision = int(geometry), int(kspace), int(precision)
        d.eta, d.alpha, d.rcut, d.kcut = float(eta), float(alpha), float(rcut), float(kcut)
        d.mesh[:] = [int(m) for m in mesh]
        d.order = int(order)
        d.alpha_build, d.rcut_build, d.kcut_build = float(alpha_build), float(rcut_build), float(kcut_build)
        d.flags = FLAG_GRAPH if graph else 0
        ex = np.ascontiguousarray(elec_xyz, dtype=np.float64)
        es = np.ascontiguousarray(elec_side, dtype=np.int8)
        sq = np.ascontiguousarray(site_q, dtype=np.float64)
        self._keep += [ex, es, sq]
        d.n_elec = ex.shape[1]
        d.elec_xyz = ex.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.elec_side = es.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
        if elec_sub is not None:
            eb = np.ascontiguousarray(elec_sub, dtype=np.uint8)
            self._keep.append(eb)
            d.elec_sub = eb.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        d.n_site = sq.shape[0]
        d.site_q = sq.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.n_elec, self.n_site = d.n_elec, d.n_site
        # the library always works on a real stream (torch's current one if
        # none is given, set once the descriptor has passed validation); every
        # call orders it after the caller's current stream and the caller's
        # current stream after it (_call)
        handle = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        r = self._lib.cpm_create(ctypes.byref(d), handle, ctypes.byref(self._ctx))
        if r != CPM_OK:
            raise CpmError(r, self._lib.cpm_last_error(None).decode())
        if stream is None:
            stream = torch.cuda.current_stream()
            self._check(self._lib.cpm_set_stream(self._ctx, ctypes.c_void_p(stream.cuda_stream)))
        self.stream = stream

    @classmethod
    def from_workload(cls, w, precision=FP64, stream=None, graph=False):
        """Context for a workloads.Workload."""
        return cls(box=w.box, geometry=GEOMETRY[w.geometry],
                   kspace=KSPACE_PPPM if w.kspace == "pppm" else KSPACE_EWALD, precision=precision,
                   eta=w.eta, alpha=w.alpha, rcut=w.rcut, kcut=w.kcut, mesh=w.mesh, order=w.order,
                   alpha_build=w.alpha_exact, rcut_build=w.rcut_exact, kcut_build=w.kcut_exact,
                   elec_xyz=w.elec_xyz, elec_side=w.elec_side, elec_sub=w.elec_sub, site_q=w.site_q,
                   stream=stream, graph=graph)

    # ---------------------------------------------------------------- calls
    def _check(self, r):
        if r != CPM_OK:
            raise CpmError(r, self._lib.cpm_last_error(self._ctx).decode())

    def _call(self, fn, *args, handle=None):
        """Run one library call with its stream ordered against the caller's.

        Inputs and outputs are tensors made or last touched on the caller's
        current stream; the library enqueues on the context's stream.  The
        context's stream first waits for the caller's stream (inputs ready,
        output memory no longer in use), and afterwards the caller's stream
        waits for the context's (results ready before the caller reads them
        or the caching allocator hands their memory out again)."""
        cur = torch.cuda.current_stream(self.stream.device)
        other = cur.cuda_stream != self.stream.cuda_stream
        if other:
            self.stream.wait_stream(cur)
        r = fn(self._ctx if handle is None else handle, *args)
        if other:
            cur.wait_stream(self.stream)
        self._check(r)

    def build_elastance(self):
        self._check(self._lib.cpm_build_elastance(self._ctx))

    def solve(self, site_xyz: torch.Tensor, dv: float, q_out=None, f_out=None, energy_out=None,
              forces=True, energy=True):
        """q* (and forces, energies) for one configuration; returns (q, f, energy) tensors."""
        dev = site_xyz.device
        if q_out is None:
            q_out = torch.empty(self.n_elec, dtype=torch.float64, device=dev)
        if forces and f_out is None:
            f_out = torch.empty((3, self.n_site), dtype=torch.float64, device=dev)
        if energy and energy_out is None:
            energy_out = torch.empty(2, dtype=torch.float64, device=dev)
        self._call(self._lib.cpm_solve, _ptr(site_xyz), float(dv), _ptr(q_out), _ptr(f_out), _ptr(energy_out))
        return q_out, f_out, energy_out

    def solve_batch(self, site_xyz: torch.Tensor, dvs, q_out=None, f_out=None, energy_out=None,
                    forces=True, energy=True):
        n_frames = site_xyz.shape[0]
        dv = np.ascontiguousarray(dvs, dtype=np.float64)
        dev = site_xyz.device
        if q_out is None:
            q_out = torch.empty((n_frames, dv.size, self.n_elec), dtype=torch.float64, device=dev)
        if forces and f_out is None:
            f_out = torch.empty((n_frames, dv.size, 3, self.n_site), dtype=torch.float64, device=dev)
        if energy and energy_out is None:
            energy_out = torch.empty((n_frames, dv.size, 2), dtype=torch.float64, device=dev)
        self._call(self._lib.cpm_solve_batch, n_frames, _ptr(site_xyz), dv.size,
                   dv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(q_out), _ptr(f_out), _ptr(energy_out))
        return q_out, f_out, energy_out

    def set_batch_shape(self, frames_per_launch: int, tiles_per_cell: int, xy_planes: int):
        """Fix the batch launch shapes (skips the tuner)."""
        self._check(self._lib.cpm_set_batch_shape(self._ctx, int(frames_per_launch), int(tiles_per_cell),
                                                  int(xy_planes)))

    def grad(self, site_xyz: torch.Tensor, dv: float, q_target: torch.Tensor):
        dev = site_xyz.device
        loss = torch.empty(1, dtype=torch.float64, device=dev)
        dldx = torch.empty((3, self.n_site), dtype=torch.float64, device=dev)
        dldv = torch.empty(1, dtype=torch.float64, device=dev)
        q = torch.empty(self.n_elec, dtype=torch.float64, device=dev)
        self._call(self._lib.cpm_grad, _ptr(site_xyz), float(dv), _ptr(q_target), _ptr(loss), _ptr(dldx),
                   _ptr(dldv), _ptr(q))
        return loss, dldx, dldv, q

    def profile(self, site_xyz: torch.Tensor, q: torch.Tensor, dv: float, n_bins: int, bulk, rho_out=None,
                psi_out=None):
        """Frame-averaged charge density and potential profile along z.

        site_xyz [F][3][n_site]; q [F][..., n_elec] (the last axis the atoms;
        a batch's q[:, v] view for one dV is accepted as it is); bulk = (z_lo,
        z_hi) window whose mean potential is zero.  Returns (rho, psi)."""
        n_frames = site_xyz.shape[0]
        if q.shape[0] != n_frames or q.shape[-1] != self.n_elec or q.stride(-1) != 1:
            raise ValueError("q must be [n_frames][..., n_elec] with contiguous atoms")
        if q.dtype != torch.float64 or not q.is_cuda:
            raise ValueError("q must be a float64 GPU tensor")
        dev = site_xyz.device
        if rho_out is None:
            rho_out = torch.empty(n_bins, dtype=torch.float64, device=dev)
        if psi_out is None:
            psi_out = torch.empty(n_bins, dtype=torch.float64, device=dev)
        self._call(self._lib.cpm_profile, n_frames, _ptr(site_xyz), ctypes.c_void_p(q.data_ptr()), q.stride(0),
                   float(dv), int(n_bins), float(bulk[0]), float(bulk[1]), _ptr(rho_out), _ptr(psi_out))
        return rho_out, psi_out

    def get_matrix(self, which: int) -> np.ndarray:
        n = self.n_elec
        out = np.empty((n, n) if which in (0, 1) else (n,), dtype=np.float64)
        self._check(self._lib.cpm_get_matrix(self._ctx, which, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def set_matrix(self, S: np.ndarray):
        S = np.ascontiguousarray(S, dtype=np.float64)
        self._check(self._lib.cpm_set_matrix(self._ctx, S.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def get_buffer(self, which: int) -> np.ndarray:
        n = self._lib.cpm_get_buffer(self._ctx, which, None)
        if n < 0:
            self._check(int(n))
        is_int = which in (BUF_CELL_START, BUF_SITE_ORDER, BUF_NCELL, BUF_BATCH_CHUNK)
        out = np.empty(int(n), dtype=np.int32 if is_int else np.float64)
        r = self._lib.cpm_get_buffer(self._ctx, which, out.ctypes.data_as(ctypes.c_void_p))
        if r < 0:
            self._check(int(r))
        return out

    def replay_kernel(self, kernel: int, reps: int):
        """Re-enqueue the last launch of one step kernel `reps` times (timing hook)."""
        self._call(self._lib.cpm_replay_kernel, int(kernel), int(reps))

    def sync_status(self) -> int:
        return int(self._lib.cpm_sync_status(self._ctx))

    def close(self):
        if self._ctx:
            self._lib.cpm_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MDLoop:
    """The constant-potential MD loop on a built Context (wraps cpm_md)."""

    def __init__(self, ctx: Context, setup):
        self.ctx = ctx
        self._lib = ctx._lib
        self._md = ctypes.c_void_p()
        self.n_groups = int(setup.n_groups)
        keep = [np.ascontiguousarray(setup.mol_size, dtype=np.int32),
                np.ascontiguousarray(setup.mol_group, dtype=np.int32),
                np.ascontiguousarray(setup.site_mass, dtype=np.float64),
                np.ascontiguousarray(setup.site_sigma, dtype=np.float64),
                np.ascontiguousarray(setup.site_eps, dtype=np.float64),
                np.ascontiguousarray(setup.lj_elec_xyz, dtype=np.float64)]
        self._keep = keep
        d = MDDesc()
        d.n_mol = keep[0].size
        d.mol_size = keep[0].ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        d.mol_group = keep[1].ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        d.n_groups = self.n_groups
        d.site_mass = keep[2].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.site_sigma = keep[3].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.site_eps = keep[4].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.n_lj_elec = keep[5].shape[1]
        d.lj_elec_xyz = keep[5].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.carbon_sigma, d.carbon_eps = float(setup.carbon_sigma), float(setup.carbon_eps)
        d.lj_cut, d.bond, d.dt = float(setup.lj_cut), float(setup.bond), float(setup.dt)
        d.temperature, d.tau, d.charge_every = float(setup.temperature), float(setup.tau), int(setup.charge_every)
        ctx._check(self._lib.cpm_md_create(ctx._ctx, ctypes.byref(d), ctypes.byref(self._md)))

    def run(self, x: torch.Tensor, v: torch.Tensor, dv: float, n_steps: int, q_out=None, thermo=True):
        """n_steps steps; x and v (device [3][n_site]) are updated in place.
        Returns (q, thermo [n_steps][4] or None)."""
        dev = x.device
        if q_out is None:
            q_out = torch.empty(self.ctx.n_elec, dtype=torch.float64, device=dev)
        th = torch.empty((n_steps, 4), dtype=torch.float64, device=dev) if thermo and n_steps > 0 else None
        self.ctx._call(self._lib.cpm_md_run, _ptr(x), _ptr(v), float(dv), int(n_steps), _ptr(q_out), _ptr(th),
                       handle=self._md)
        return q_out, th

    def set_thermostat(self, on: bool):
        self._lib.cpm_md_set_thermostat(self._md, 1 if on else 0)

    def state(self):
        xi = np.zeros(self.n_groups)
        eta = np.zeros(self.n_groups)
        step = ctypes.c_longlong()
        self.ctx._check(self._lib.cpm_md_state(self._md, xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               eta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               ctypes.byref(step)))
        return xi, eta, int(step.value)

    def close(self):
        if self._md:
            self._lib.cpm_md_destroy(self._md)
            self._md = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
