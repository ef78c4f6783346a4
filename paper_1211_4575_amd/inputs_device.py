"""ctypes binding of libpp_inputs.so: on-device twins of the host loaders in inputs.py, for
workloads too large to generate on the host (input generation only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpp_inputs.so")
_lib = None

FP64, SPLIT_NEAREST, SPLIT_FLOOR = 0, 1, 2


def split_mode(split: bool, shape_order: int) -> int:
    """Generator output mode for a run: FP64 positions, or the split form whose offset
    convention goes with the weight order (nearest node for quadratic, node below for cubic)."""
    if not split:
        return FP64
    return SPLIT_NEAREST if shape_order == 2 else SPLIT_FLOOR


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1211_4575_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.ppi_philox_blocks.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
                                        ctypes.c_int64, vp, vp]
        L.ppi_philox_blocks.restype = ctypes.c_int
        L.ppi_pair_maxwell_juttner.argtypes = [ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64,
                                               ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                               ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        L.ppi_pair_maxwell_juttner.restype = ctypes.c_int
        L.ppi_two_stream_lattice.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int32), ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                             ctypes.POINTER(vp), vp]
        L.ppi_two_stream_lattice.restype = ctypes.c_int
        L.ppi_kelvin_helmholtz.argtypes = [ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                           ctypes.POINTER(vp), vp]
        L.ppi_kelvin_helmholtz.restype = ctypes.c_int
        L.ppi_mmi.argtypes = [ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, ctypes.c_int64,
                              ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.POINTER(vp),
                              ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        L.ppi_mmi.restype = ctypes.c_int
        _lib = L
    return _lib


def philox_blocks(seed, block, stream, ctr0, count, out, hip_stream):
    """out: int32/uint32 torch tensor of 4*count elements on the device."""
    rc = lib().ppi_philox_blocks(seed, block, stream, ctr0, count, out.data_ptr(), hip_stream)
    if rc:
        raise RuntimeError(f"ppi_philox_blocks failed ({rc})")


def pair_maxwell_juttner(seed, n, start, count, theta, split, cells, offs, us, hip_stream):
    """cells: [cell_e, cell_p] int32 tensors (split) or None; offs/us: [[3 tensors] x 2];
    writes particle indices [start, start+count) into element 0.. of each tensor."""
    vp = ctypes.c_void_p
    n_arr = (ctypes.c_int32 * 3)(*[int(v) for v in n])
    cell_arr = (vp * 2)(*([c.data_ptr() for c in cells] if cells is not None else [None, None]))
    off_arr = (vp * 6)(*[offs[s][d].data_ptr() for s in range(2) for d in range(3)])
    u_arr = (vp * 6)(*[us[s][d].data_ptr() for s in range(2) for d in range(3)])
    rc = lib().ppi_pair_maxwell_juttner(seed, n_arr, start, count, theta, int(split), cell_arr, off_arr, u_arr,
                                        hip_stream)
    if rc:
        raise RuntimeError(f"ppi_pair_maxwell_juttner failed ({rc})")


def two_stream_lattice(seed, wl, n, per_dim, v_beam, uth, split, cells, offs, us, hip_stream):
    """Quiet-lattice two-beam load written into device tensors (see inputs.two_stream)."""
    vp = ctypes.c_void_p
    n_arr = (ctypes.c_int32 * 3)(*[int(v) for v in n])
    k_arr = (ctypes.c_int32 * 3)(*[int(v) for v in per_dim])
    cell_arr = (vp * 2)(*([c.data_ptr() for c in cells] if cells is not None else [None, None]))
    off_arr = (vp * 6)(*[offs[s][d].data_ptr() for s in range(2) for d in range(3)])
    u_arr = (vp * 6)(*[us[s][d].data_ptr() for s in range(2) for d in range(3)])
    rc = lib().ppi_two_stream_lattice(seed, wl, n_arr, k_arr, v_beam, uth, int(split), cell_arr, off_arr, u_arr,
                                      hip_stream)
    if rc:
        raise RuntimeError(f"ppi_two_stream_lattice failed ({rc})")


def kelvin_helmholtz(seed, n, start, count, v0, width, uth, split, cells, offs, us, hip_stream):
    """Shear-layer load of particle indices [start, start + count) into device tensors (see
    inputs.kelvin_helmholtz)."""
    vp = ctypes.c_void_p
    n_arr = (ctypes.c_int32 * 3)(*[int(v) for v in n])
    cell_arr = (vp * 2)(*([c.data_ptr() for c in cells] if cells is not None else [None, None]))
    off_arr = (vp * 6)(*[offs[s][d].data_ptr() for s in range(2) for d in range(3)])
    u_arr = (vp * 6)(*[us[s][d].data_ptr() for s in range(2) for d in range(3)])
    rc = lib().ppi_kelvin_helmholtz(seed, n_arr, start, count, v0, width, uth, int(split), cell_arr, off_arr, u_arr,
                                    hip_stream)
    if rc:
        raise RuntimeError(f"ppi_kelvin_helmholtz failed ({rc})")


def mmi(seed, n, start, count, gamma_b, T_b, T_p, mass_ratio, split, cells, offs, us, hip_stream, quiet=False,
        lattice=None):
    """Mixed-mode two-stream load of particle indices [start, start+count) of four species
    (see inputs.mmi, ``quiet`` and ``lattice`` its quiet start and lattice positions) into
    device tensors: cells [4] int32 (split) or None, offs/us [[3] x 4]."""
    vp = ctypes.c_void_p
    n_arr = (ctypes.c_int32 * 3)(*[int(v) for v in n])
    cell_arr = (vp * 4)(*([c.data_ptr() for c in cells] if cells is not None else [None] * 4))
    off_arr = (vp * 12)(*[offs[s][d].data_ptr() for s in range(4) for d in range(3)])
    u_arr = (vp * 12)(*[us[s][d].data_ptr() for s in range(4) for d in range(3)])
    lat = (ctypes.c_int32 * 3)(*[int(v) for v in lattice]) if lattice is not None else None
    rc = lib().ppi_mmi(seed, n_arr, start, count, gamma_b, T_b, T_p, mass_ratio, int(bool(quiet)), lat, int(split),
                       cell_arr, off_arr, u_arr, hip_stream)
    if rc:
        raise RuntimeError(f"ppi_mmi failed ({rc})")
