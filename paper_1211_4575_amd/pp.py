"""Thin ctypes binding of libpp (include/pp.h).

The functions carry the C names and only marshal arguments; every step of the particle
step runs in the HIP kernels of libpp.so.  Device memory and streams come from PyTorch.
There is no fallback: if libpp.so is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpp.so")

PP_OK, PP_E_ARG, PP_E_CFL, PP_E_NONFINITE, PP_E_NOCONV, PP_E_CAPACITY, PP_E_HIP, PP_E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
PP_PREC_FP64, PP_PREC_FP32_SPLIT = 0, 1
PP_PUSH_VAY, PP_PUSH_BORIS = 0, 1
PP_CURRENT_CC, PP_CURRENT_DIRECT = 0, 1
PP_MAX_SPECIES = 8
PP_FLAG_CFL, PP_FLAG_NONFINITE, PP_FLAG_OUT_OF_TILE = 1, 2, 4
PP_DIAG_MOMENTS, PP_DIAG_FIELDS, PP_DIAG_RHO, PP_DIAG_DIVB, PP_DIAG_RELAX, PP_DIAG_ALL = 1, 2, 4, 8, 16, 31

EXPORTED = ("pp_workspace_size", "pp_create", "pp_init_species", "pp_gather_push_deposit", "pp_field_step", "pp_sort_particles",
            "pp_step",
            "pp_diagnostics", "pp_get_particles", "pp_timing_enable", "pp_timing_read", "pp_destroy",
            "pp_status_str", "pp_last_hip_error", "pp_batch_create", "pp_batch_add", "pp_batch_remove",
            "pp_batch_size", "pp_batch_step", "pp_batch_destroy", "pp_batch_step_noalloc")


class pp_params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("d", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("c", ctypes.c_double),
        ("eps0", ctypes.c_double),
        ("shape_order", ctypes.c_int32),
        ("field_order", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("pusher", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("relax_tol", ctypes.c_double),
        ("relax_max_iter", ctypes.c_int32),
        ("rho_background", ctypes.c_double),
        ("rad_tau", ctypes.c_double),
        ("current_scheme", ctypes.c_int32),
        ("gauss_filter_passes", ctypes.c_int32),
        ("time_order", ctypes.c_int32),
        ("gauss_filter_every", ctypes.c_int32),
    ]


class pp_mesh(ctypes.Structure):
    _fields_ = [("E", ctypes.c_void_p), ("B", ctypes.c_void_p), ("J", ctypes.c_void_p)]


class pp_particles(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("cell", ctypes.c_void_p),
        ("pos", ctypes.c_void_p * 3),
        ("u", ctypes.c_void_p * 3),
        ("id", ctypes.c_void_p),
        ("cell_alt", ctypes.c_void_p),
        ("pos_alt", ctypes.c_void_p * 3),
        ("u_alt", ctypes.c_void_p * 3),
        ("id_alt", ctypes.c_void_p),
    ]


class pp_diag(ctypes.Structure):
    _fields_ = [
        ("kinetic", ctypes.c_double * PP_MAX_SPECIES),
        ("momentum", (ctypes.c_double * 3) * PP_MAX_SPECIES),
        ("field_E", ctypes.c_double),
        ("field_B", ctypes.c_double),
        ("field_Ex", ctypes.c_double),
        ("gauss_max", ctypes.c_double),
        ("cc_max", ctypes.c_double),
        ("rho_ref", ctypes.c_double),
        ("divB_max", ctypes.c_double),
        ("relax_resid", ctypes.c_double),
        ("relax_iters", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("step", ctypes.c_int64),
        ("relax_resid_meas", ctypes.c_double),
    ]


_lib = None


class PPError(RuntimeError):
    def __init__(self, where: str, status: int):
        L = lib()
        msg = L.pp_status_str(status).decode()
        hip = L.pp_last_hip_error().decode()
        super().__init__(f"{where}: {msg} ({status}){' / ' + hip if hip else ''}")
        self.status = status


def lib():
    """Load libpp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1211_4575_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.pp_workspace_size.argtypes = [ctypes.POINTER(pp_params), ctypes.c_int64, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_size_t)]
        L.pp_create.argtypes = [ctypes.POINTER(pp_params), ctypes.POINTER(pp_mesh), vp, ctypes.POINTER(vp)]
        L.pp_init_species.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.POINTER(pp_particles)]
        L.pp_gather_push_deposit.argtypes = [vp]
        L.pp_field_step.argtypes = [vp]
        L.pp_sort_particles.argtypes = [vp, ctypes.c_int32]
        L.pp_step.argtypes = [vp]
        L.pp_diagnostics.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(pp_diag)]
        L.pp_get_particles.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(pp_particles)]
        L.pp_timing_enable.argtypes = [vp, ctypes.c_int32]
        L.pp_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.pp_destroy.argtypes = [vp]
        L.pp_batch_create.argtypes = [ctypes.c_int32, vp, ctypes.POINTER(vp)]
        L.pp_batch_add.argtypes = [vp, vp]
        L.pp_batch_remove.argtypes = [vp, vp]
        L.pp_batch_size.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.pp_batch_step.argtypes = [vp]
        L.pp_batch_step_noalloc.argtypes = [vp]
        L.pp_batch_destroy.argtypes = [vp]
        L.pp_status_str.argtypes = [ctypes.c_int32]
        L.pp_status_str.restype = ctypes.c_char_p
        L.pp_last_hip_error.argtypes = []
        L.pp_last_hip_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("pp_status_str", "pp_last_hip_error"):
                getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(where, st):
    if st != PP_OK:
        raise PPError(where, st)


# ---- the C calls, same names ------------------------------------------------------------
def pp_workspace_size(params: pp_params, max_particles: int, nspecies: int) -> int:
    b = ctypes.c_size_t()
    _check("pp_workspace_size", lib().pp_workspace_size(ctypes.byref(params), int(max_particles), int(nspecies),
                                                        ctypes.byref(b)))
    return b.value


def pp_create(params: pp_params, mesh: pp_mesh, stream: int) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check("pp_create", lib().pp_create(ctypes.byref(params), ctypes.byref(mesh), ctypes.c_void_p(stream),
                                        ctypes.byref(h)))
    return h


def pp_init_species(run, s, q, m, w, parts: pp_particles):
    _check("pp_init_species", lib().pp_init_species(run, s, q, m, w, ctypes.byref(parts)))


def pp_gather_push_deposit(run):
    _check("pp_gather_push_deposit", lib().pp_gather_push_deposit(run))


def pp_field_step(run):
    _check("pp_field_step", lib().pp_field_step(run))


def pp_sort_particles(run, s=-1):
    _check("pp_sort_particles", lib().pp_sort_particles(run, s))


def pp_step(run):
    _check("pp_step", lib().pp_step(run))


def pp_diagnostics(run, what=PP_DIAG_ALL) -> pp_diag:
    d = pp_diag()
    _check("pp_diagnostics", lib().pp_diagnostics(run, what, ctypes.byref(d)))
    return d


def pp_get_particles(run, s) -> pp_particles:
    p = pp_particles()
    _check("pp_get_particles", lib().pp_get_particles(run, s, ctypes.byref(p)))
    return p


def pp_timing_enable(run, enable=True):
    _check("pp_timing_enable", lib().pp_timing_enable(run, int(bool(enable))))


def pp_timing_read(run):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check("pp_timing_read", lib().pp_timing_read(run, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def pp_destroy(run):
    _check("pp_destroy", lib().pp_destroy(run))


def pp_batch_create(max_runs: int, stream: int):
    h = ctypes.c_void_p()
    _check("pp_batch_create", lib().pp_batch_create(int(max_runs), ctypes.c_void_p(stream), ctypes.byref(h)))
    return h


def pp_batch_add(batch, run):
    _check("pp_batch_add", lib().pp_batch_add(batch, run))


def pp_batch_remove(batch, run):
    _check("pp_batch_remove", lib().pp_batch_remove(batch, run))


def pp_batch_size(batch) -> int:
    n = ctypes.c_int32()
    _check("pp_batch_size", lib().pp_batch_size(batch, ctypes.byref(n)))
    return n.value


def pp_batch_step(batch):
    _check("pp_batch_step", lib().pp_batch_step(batch))


def pp_batch_step_noalloc(batch):
    _check("pp_batch_step_noalloc", lib().pp_batch_step_noalloc(batch))


def pp_batch_destroy(batch):
    _check("pp_batch_destroy", lib().pp_batch_destroy(batch))


# ---- convenience owner of the torch tensors ---------------------------------------------
def make_params(n, d=(1.0, 1.0, 1.0), dt=0.4, c=1.0, eps0=1.0, shape_order=2, field_order=2, alpha=0.55,
                pusher=0, precision=PP_PREC_FP64, relax_tol=1e-14, relax_max_iter=200, rho_background=0.0,
                rad_tau=0.0, current_scheme=0, gauss_filter_passes=0, time_order=2, gauss_filter_every=1):
    p = pp_params()
    p.n[:] = [int(v) for v in n]
    p.d[:] = [float(v) for v in d]
    p.dt, p.c, p.eps0 = float(dt), float(c), float(eps0)
    p.shape_order, p.field_order = int(shape_order), int(field_order)
    p.alpha, p.pusher, p.precision = float(alpha), int(pusher), int(precision)
    p.relax_tol, p.relax_max_iter = float(relax_tol), int(relax_max_iter)
    p.rho_background = float(rho_background)
    p.rad_tau = float(rad_tau)
    p.current_scheme, p.gauss_filter_passes = int(current_scheme), int(gauss_filter_passes)
    p.time_order = int(time_order)
    p.gauss_filter_every = int(gauss_filter_every)
    return p


class Run:
    """One PIC run on the GPU: torch owns the mesh and particle memory, libpp computes.

    ``species``: list of dicts with q, m, w and either ``pos`` [3, n] float64 positions (cell
    units) or, for the split form, ``cell`` int32 + ``off`` [3, n] float32; ``u`` [3, n].
    """

    def __init__(self, params: pp_params, species, E=None, B=None, device="cuda:0", with_id=True):
        import torch

        lib()
        self.torch = torch
        self.dev = torch.device(device)
        self.params = params
        self.split = params.precision == PP_PREC_FP32_SPLIT
        nx, ny, nz = params.n
        shape = (3, nz, ny, nx)
        f64 = torch.float64
        self.E = torch.zeros(shape, dtype=f64, device=self.dev) if E is None else torch.as_tensor(
            np.ascontiguousarray(E), dtype=f64).to(self.dev)
        self.B = torch.zeros(shape, dtype=f64, device=self.dev) if B is None else torch.as_tensor(
            np.ascontiguousarray(B), dtype=f64).to(self.dev)
        self.J = torch.zeros(shape, dtype=f64, device=self.dev)
        self.mesh = pp_mesh(self.E.data_ptr(), self.B.data_ptr(), self.J.data_ptr())
        self.stream = torch.cuda.current_stream(self.dev)
        self.handle = pp_create(params, self.mesh, self.stream.cuda_stream)
        self.bufs = []
        self.species = []
        for s, sp in enumerate(species):
            self._add_species(s, sp, with_id)

    def _add_species(self, s, sp, with_id):
        torch = self.torch
        rt = torch.float32 if self.split else torch.float64
        if isinstance(sp.get("u"), torch.Tensor):
            # device tensors handed over as they are
            cell = sp.get("cell")
            pos = sp["off"] if self.split else sp["pos"]
            u = sp["u"]
            assert u.dtype == rt and pos.dtype == rt and u.is_contiguous() and pos.is_contiguous()
            assert cell is None or (cell.dtype == torch.int32 and cell.is_contiguous())
        elif self.split:
            cell = torch.as_tensor(np.ascontiguousarray(sp["cell"], dtype=np.int32)).to(self.dev)
            pos = torch.as_tensor(np.ascontiguousarray(sp["off"], dtype=np.float32)).to(self.dev)
            u = torch.as_tensor(np.ascontiguousarray(sp["u"])).to(dtype=rt, device=self.dev).contiguous()
        else:
            cell = None
            pos = torch.as_tensor(np.ascontiguousarray(sp["pos"], dtype=np.float64)).to(self.dev)
            u = torch.as_tensor(np.ascontiguousarray(sp["u"])).to(dtype=rt, device=self.dev).contiguous()
        n = pos.shape[1]
        ids = torch.arange(n, dtype=torch.int64, device=self.dev) if with_id else None
        alt = dict(pos=torch.empty_like(pos), u=torch.empty_like(u),
                   cell=torch.empty_like(cell) if cell is not None else None,
                   id=torch.empty_like(ids) if ids is not None else None)
        keep = dict(pos=pos, u=u, cell=cell, id=ids, alt=alt)
        self.bufs.append(keep)
        P = pp_particles()
        P.n = n
        ptr = lambda t: t.data_ptr() if t is not None else None
        P.cell = ptr(cell)
        P.cell_alt = ptr(alt["cell"])
        P.id = ptr(ids)
        P.id_alt = ptr(alt["id"])
        for d in range(3):
            P.pos[d] = pos[d].data_ptr()
            P.u[d] = u[d].data_ptr()
            P.pos_alt[d] = alt["pos"][d].data_ptr()
            P.u_alt[d] = alt["u"][d].data_ptr()
        pp_init_species(self.handle, s, float(sp["q"]), float(sp["m"]), float(sp["w"]), P)
        self.species.append(dict(q=float(sp["q"]), m=float(sp["m"]), w=float(sp["w"]), n=n))

    # -- the step, in the paper's order --
    def gather_push_deposit(self):
        pp_gather_push_deposit(self.handle)

    def sort(self, s=-1):
        pp_sort_particles(self.handle, s)

    def field_step(self):
        pp_field_step(self.handle)

    def step(self, sort=True):
        if self.params.time_order == 4:  # the composed step (three substeps) in the library
            pp_step(self.handle)
            return
        self.gather_push_deposit()
        if sort or self.split:
            self.sort()
        self.field_step()

    def diagnostics(self, what=PP_DIAG_ALL) -> pp_diag:
        return pp_diagnostics(self.handle, what)

    # -- readback helpers (tests) --
    def _wrap_ptr(self, ptr, n, dtype):
        """Find which owned tensor a raw device pointer belongs to."""
        torch = self.torch
        for b in self.bufs:
            for t in (b["pos"], b["u"], b["cell"], b["id"], b["alt"]["pos"], b["alt"]["u"], b["alt"]["cell"],
                      b["alt"]["id"]):
                if t is None:
                    continue
                if t.dim() == 2:
                    for d in range(t.shape[0]):
                        if t[d].data_ptr() == ptr:
                            return t[d]
                elif t.data_ptr() == ptr:
                    return t
        raise KeyError(ptr)

    def particles(self, s):
        """Current particle state of species s as numpy arrays (synchronises)."""
        P = pp_get_particles(self.handle, s)
        self.torch.cuda.synchronize(self.dev)
        n = P.n
        if n == 0:  # an empty species may hold no buffers at all
            rt = np.float32 if self.split else np.float64
            out = dict(u=np.zeros((3, 0), rt), pos=np.zeros((3, 0), rt))
            if self.split:
                out["cell"] = np.zeros(0, np.int32)
            if self.bufs[s]["id"] is not None:
                out["id"] = np.zeros(0, np.int64)
            return out
        out = dict(u=np.stack([self._wrap_ptr(P.u[d], n, None).cpu().numpy() for d in range(3)]))
        out["pos"] = np.stack([self._wrap_ptr(P.pos[d], n, None).cpu().numpy() for d in range(3)])
        if self.split:
            out["cell"] = self._wrap_ptr(P.cell, n, None).cpu().numpy()
        if P.id:
            out["id"] = self._wrap_ptr(P.id, n, None).cpu().numpy()
        return out

    def particle_tensors(self, s):
        """Current particle state of species s as device tensors: views of the run's own
        buffers (no copy), valid until the next step or sort."""
        P = pp_get_particles(self.handle, s)
        n = P.n
        if n == 0:
            return {k: (v if k in ("cell", "id") else [v[d] for d in range(3)]) if v is not None else None
                    for k, v in self.bufs[s].items() if k != "alt"}
        out = dict(u=[self._wrap_ptr(P.u[d], n, None) for d in range(3)],
                   pos=[self._wrap_ptr(P.pos[d], n, None) for d in range(3)])
        out["cell"] = self._wrap_ptr(P.cell, n, None) if self.split else None
        out["id"] = self._wrap_ptr(P.id, n, None) if P.id else None
        return out

    def fields(self):
        self.torch.cuda.synchronize(self.dev)
        return self.E.cpu().numpy(), self.B.cpu().numpy(), self.J.cpu().numpy()

    def timing(self, enable=True):
        pp_timing_enable(self.handle, enable)

    def timing_read(self):
        return pp_timing_read(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            pp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
