"""Python binding of libetpic (ctypes): argument marshalling only.

Every step of the particle path runs in the HIP kernels of libetpic.so; this
module converts torch tensors (device memory, streams) into the plain pointers
of the C ABI declared in include/etpic.h.  If the library is missing, every
entry point raises: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libetpic.so")

OK, EINVAL, ESTATE, EHIP, EMESH, EPARTICLE, EWALK, ENAN, ENOCONV, EIO = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
FP64, MIXED, MIXED_FIXED = 0, 1, 2
DEV_HOPCAP, DEV_NAN, DEV_BADTET = 1, 2, 4
STEP_XCD_REMAP = 1
STEP_TIMING = 2
STEP_TIMING_ALL = 256
STEP_SLICES_1, STEP_SLICES_4, STEP_SLICES_16 = 4, 8, 16
STEP_SLICES_2 = 512
STEP_WALK_BY_SLICE = 32
NS_WARM = 64
EM_SPLIT = 128
HOP_CAP = 64

EXPORTS = (
    "etpic_last_error", "etpic_create", "etpic_destroy", "etpic_workspace_bytes", "etpic_workspace_bind",
    "etpic_mesh_sizes", "etpic_mesh_upload", "etpic_mesh_canonical",
    "etpic_mesh_counts", "etpic_mesh_edges", "etpic_mesh_faces", "etpic_gather_push_deposit", "etpic_sort",
    "etpic_vertex_charge", "etpic_gauss_residual", "etpic_gauss_residual_noalloc", "etpic_stream_probe",
    "etpic_last_push_slices", "etpic_kernel_time",
    "etpic_check",
    "etpic_adjoint_workspace", "etpic_forward_checkpointed", "etpic_backward",
    "etpic_field_bytes", "etpic_field_setup", "etpic_field_nnz", "etpic_field_spmv", "etpic_field_step",
    "etpic_particles_locate", "etpic_particles_positions", "etpic_coarse_step", "etpic_run_steps",
    "etpic_sort_run_steps", "etpic_ds_rows_bytes", "etpic_ds_rows_bind", "etpic_ds_history_bytes", "etpic_ds_steps", "etpic_ds_sort",
    "etpic_ns_bytes", "etpic_ns_setup", "etpic_ns_info", "etpic_ns_solve", "etpic_ns_run_steps", "etpic_ns_correct", "etpic_em_steps",
    "etpic_sol_source",
    "etpic_qh_last_error", "etpic_qh_create", "etpic_qh_bytes", "etpic_qh_bind", "etpic_qh_destroy", "etpic_qh_counts", "etpic_qh_project_b",
    "etpic_qh_project_e", "etpic_tree_cotree", "etpic_checkpoint_write", "etpic_checkpoint_info",
    "etpic_checkpoint_read", "etpic_cotree_create", "etpic_cotree_bytes", "etpic_cotree_bind", "etpic_cotree_destroy",
    "etpic_cotree_counts", "etpic_cotree_apply", "etpic_cotree_b_field", "etpic_cotree_step",
)


def checkpoint_info(path):
    """Header of a particle checkpoint file (host only): n, precision, step,
    has_id."""
    n, step = C.c_int64(0), C.c_int64(0)
    prec, has_id = C.c_int(0), C.c_int(0)
    _chk(lib().etpic_checkpoint_info(os.fsencode(path), C.byref(n), C.byref(prec), C.byref(step), C.byref(has_id)))
    return {"n": int(n.value), "precision": int(prec.value), "step": int(step.value), "has_id": bool(has_id.value)}


class EtpicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"etpic error {code}: {msg}")
        self.code = code


class _Particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("lam", C.c_void_p * 3), ("vel", C.c_void_p * 3), ("tet", C.c_void_p),
                ("id", C.c_void_p)]


class _Fields(C.Structure):
    _fields_ = [("e_env", C.c_void_p), ("e_dc", C.c_void_p), ("b_env", C.c_void_p), ("b_dc", C.c_void_p)]


class _Species(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("w", C.c_double)]


_lib = None


def lib():
    """Load libetpic.so (built in-tree by build.py); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libetpic.so not built ({LIB_PATH}); run paper_2208_12795_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, i64p, i32p, dp = C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double)
    L.etpic_last_error.restype = C.c_char_p
    L.etpic_create.argtypes = [C.POINTER(vp), C.c_int]
    L.etpic_destroy.argtypes = [vp]
    szp = C.POINTER(C.c_size_t)
    L.etpic_workspace_bytes.argtypes = [szp]
    L.etpic_workspace_bind.argtypes = [vp, vp, C.c_size_t]
    L.etpic_mesh_sizes.argtypes = [C.c_int64, dp, C.c_int64, i32p, i64p, szp]
    L.etpic_mesh_upload.argtypes = [vp, C.c_int64, dp, C.c_int64, i32p, vp, C.c_size_t]
    L.etpic_field_bytes.argtypes = [vp, C.c_double, C.c_double, szp]
    L.etpic_ns_bytes.argtypes = [vp, C.c_double, szp]
    L.etpic_ds_rows_bytes.argtypes = [vp, szp]
    L.etpic_ds_rows_bind.argtypes = [vp, vp, C.c_size_t]
    L.etpic_qh_bytes.argtypes = [vp, szp]
    L.etpic_qh_bind.argtypes = [vp, vp, C.c_size_t]
    L.etpic_mesh_canonical.argtypes = [C.c_int64, dp, C.c_int64, i32p, i64p, i32p, i32p]
    L.etpic_mesh_counts.argtypes = [vp, i64p]
    L.etpic_mesh_edges.argtypes = [vp, i32p]
    L.etpic_mesh_faces.argtypes = [vp, i32p]
    L.etpic_gather_push_deposit.argtypes = [vp, C.POINTER(_Particles), C.c_int, C.POINTER(_Species),
                                            C.POINTER(_Fields), C.c_int64, C.c_double, C.c_double, vp, vp,
                                            C.c_uint32, vp]
    L.etpic_sort.argtypes = [vp, C.POINTER(_Particles), C.POINTER(_Particles), C.c_int, vp]
    L.etpic_vertex_charge.argtypes = [vp, C.POINTER(_Particles), C.c_int, C.POINTER(_Species), vp, vp]
    L.etpic_gauss_residual.argtypes = [vp, vp, vp, vp, dp, vp]
    L.etpic_gauss_residual_noalloc.argtypes = [vp, vp, vp, vp, dp, vp]
    L.etpic_stream_probe.argtypes = [vp, C.POINTER(_Particles), C.c_int, C.c_uint32, vp]
    L.etpic_last_push_slices.argtypes = [vp, C.POINTER(C.c_int)]
    L.etpic_kernel_time.argtypes = [vp, dp, i64p, C.c_int]
    L.etpic_adjoint_workspace.argtypes = [vp, C.c_int64, C.c_int, C.c_int, C.POINTER(C.c_size_t)]
    L.etpic_forward_checkpointed.argtypes = [vp, C.POINTER(_Particles), C.POINTER(_Species), C.POINTER(_Fields),
                                             C.c_int64, C.c_int, C.c_double, C.c_double, C.c_int, vp, C.c_size_t,
                                             vp, vp]
    L.etpic_backward.argtypes = [vp, C.c_int64, C.POINTER(_Species), C.POINTER(_Fields), C.c_int64, C.c_int,
                                 C.c_double, C.c_double, C.c_int, vp, C.c_size_t, C.c_void_p * 3, C.c_void_p * 3,
                                 vp, vp]
    L.etpic_check.argtypes = [vp, vp, C.POINTER(C.c_uint32)]
    L.etpic_checkpoint_write.argtypes = [vp, C.POINTER(_Particles), C.c_int, C.c_int64, C.c_char_p, vp]
    L.etpic_checkpoint_info.argtypes = [C.c_char_p, i64p, C.POINTER(C.c_int), i64p, C.POINTER(C.c_int)]
    L.etpic_checkpoint_read.argtypes = [vp, C.POINTER(_Particles), C.c_int, C.c_char_p, i64p, vp]
    L.etpic_particles_locate.argtypes = [vp, C.POINTER(_Particles), C.c_int, C.c_void_p * 3, vp, vp]
    L.etpic_particles_positions.argtypes = [vp, C.POINTER(_Particles), C.c_int, C.c_void_p * 3, vp]
    L.etpic_run_steps.argtypes = [vp, C.POINTER(_Particles), C.c_int, C.POINTER(_Species), C.POINTER(_Fields),
                                  C.c_int64, C.c_int, C.c_double, C.c_double, vp, vp, C.c_uint32, vp]
    L.etpic_ds_history_bytes.argtypes = [C.c_int64, C.c_int, C.POINTER(C.c_size_t)]
    L.etpic_ds_sort.argtypes = [vp, C.POINTER(_Particles), C.POINTER(_Particles), C.c_int, vp, vp, C.c_size_t, vp]
    L.etpic_ds_steps.argtypes = [vp, C.POINTER(_Particles), C.c_int, vp, C.c_size_t, C.POINTER(_Species), C.POINTER(_Fields),
                                 C.c_int64, C.c_int, C.c_int, C.c_double, C.c_double, vp, vp, C.c_uint32, vp]
    L.etpic_sort_run_steps.argtypes = [vp, C.POINTER(_Particles), C.POINTER(_Particles), C.c_int,
                                       C.POINTER(_Species), C.POINTER(_Fields), C.c_int64, C.c_int, C.c_double,
                                       C.c_double, vp, vp, C.c_uint32, vp]
    L.etpic_coarse_step.argtypes = [vp, C.POINTER(_Particles), C.c_int, C.POINTER(_Species), _Fields * 3,
                                    C.c_double, C.c_double, C.c_int, C.c_double, vp, vp, C.c_uint32, vp]
    L.etpic_field_setup.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double, vp, C.c_size_t]
    L.etpic_field_nnz.argtypes = [vp, i64p]
    L.etpic_field_spmv.argtypes = [vp, vp, vp, C.c_double, C.c_double, C.c_double, vp]
    L.etpic_field_step.argtypes = [vp, C.c_double, vp, vp, vp, vp, vp, C.c_double, C.c_int, C.POINTER(C.c_int),
                                   dp, vp]
    L.etpic_ns_setup.argtypes = [vp, C.c_double, vp, C.c_size_t]
    L.etpic_ns_info.argtypes = [vp, i64p, i64p]
    L.etpic_ns_solve.argtypes = [vp, vp, vp, C.c_double, C.c_double, vp, vp, C.c_double, C.c_int, C.c_uint32,
                                 C.POINTER(C.c_int), dp, vp]
    L.etpic_ns_run_steps.argtypes = [vp, vp, C.c_int, vp, vp, C.c_int64, C.c_int, C.c_int, C.c_double, C.c_double,
                                     vp, vp, vp, C.c_double, C.c_int, C.c_uint32, C.POINTER(C.c_int), vp]
    L.etpic_ns_correct.argtypes = [vp, vp, vp, C.c_double, C.c_double, vp, vp, C.c_double, C.c_int, C.c_uint32,
                                   C.POINTER(C.c_int), dp, vp]
    L.etpic_sol_source.argtypes = [vp, vp, vp, C.c_double, C.c_int, C.c_uint32, C.POINTER(C.c_int), dp, vp]
    L.etpic_em_steps.argtypes = [vp, vp, C.c_int, vp, C.c_int64, C.c_int, vp, vp, vp, vp, vp, vp, vp, vp, C.c_double,
                                 C.c_int, C.c_uint32, C.POINTER(C.c_int), vp]
    L.etpic_qh_last_error.restype = C.c_char_p
    L.etpic_qh_last_error.argtypes = []
    L.etpic_qh_create.argtypes = [C.POINTER(vp), C.c_int, C.c_int64, dp, C.c_int64, i32p, C.c_double]
    L.etpic_qh_destroy.argtypes = [vp]
    L.etpic_qh_destroy.restype = None
    L.etpic_qh_counts.argtypes = [vp, i64p]
    L.etpic_qh_project_b.argtypes = [vp, vp, vp, C.c_double, C.c_int, C.POINTER(C.c_int), dp, vp]
    L.etpic_qh_project_e.argtypes = [vp, vp, vp, vp, vp, C.c_double, C.c_int, C.POINTER(C.c_int), dp, vp]
    L.etpic_tree_cotree.argtypes = [C.c_int64, dp, C.c_int64, i32p, C.POINTER(C.c_uint8), C.POINTER(C.c_uint8),
                                    i64p]
    L.etpic_cotree_create.argtypes = [C.POINTER(vp), vp, C.c_int64, dp, C.c_int64, i32p, C.c_double]
    L.etpic_cotree_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.etpic_cotree_bind.argtypes = [vp, vp, C.c_size_t]
    L.etpic_cotree_destroy.argtypes = [vp]
    L.etpic_cotree_destroy.restype = None
    L.etpic_cotree_counts.argtypes = [vp, i64p]
    L.etpic_cotree_apply.argtypes = [vp, vp, C.c_int, vp, vp, C.c_double, C.c_int, vp]
    L.etpic_cotree_b_field.argtypes = [vp, vp, vp, vp, C.c_double, C.c_int, vp]
    L.etpic_cotree_step.argtypes = [vp, vp, C.c_double, C.c_double, vp, vp, vp, C.c_double, C.c_int, C.c_double,
                                    C.c_int, C.POINTER(C.c_int), dp, vp]
    for name in EXPORTS:
        if name in ("etpic_qh_last_error", "etpic_qh_destroy", "etpic_cotree_destroy"):
            continue
        if name != "etpic_last_error":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _chk(rc):
    if rc != OK:
        raise EtpicError(rc, lib().etpic_last_error().decode())
    return rc


def _np_ptr(a, ty):
    return a.ctypes.data_as(C.POINTER(ty))


def _dptr(t):
    """device pointer of a torch tensor (None -> NULL)"""
    return None if t is None else C.c_void_p(t.data_ptr())


def _vec(t, n, name, dtype="float64", optional=True):
    """Device pointer of t after checking that it is a contiguous CUDA tensor
    of `dtype` holding exactly n elements (the library reads and writes that
    many through the pointer); None -> NULL when optional (the library then
    decides whether NULL is allowed).  A mismatch raises EtpicError(EINVAL)
    before anything is launched."""
    import torch
    if t is None:
        if optional:
            return None
        raise EtpicError(EINVAL, f"{name} is required")
    want = getattr(torch, dtype)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise EtpicError(EINVAL, f"{name} must be a CUDA tensor")
    if t.dtype != want:
        raise EtpicError(EINVAL, f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise EtpicError(EINVAL, f"{name} must be contiguous")
    if t.numel() != n:
        raise EtpicError(EINVAL, f"{name} must hold {n} elements, got {t.numel()} (shape {tuple(t.shape)})")
    return C.c_void_p(t.data_ptr())


def _rows3(t, n, name, dtype="float64"):
    """The three row pointers of a contiguous [3, n] CUDA tensor of `dtype`."""
    _vec(t, 3 * n, name, dtype, optional=False)
    if t.dim() != 2 or t.shape[0] != 3:
        raise EtpicError(EINVAL, f"{name} must have shape [3, {n}], got {tuple(t.shape)}")
    return (C.c_void_p * 3)(*[t[k].data_ptr() for k in range(3)])


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def mesh_canonical(xyz, tet_vert):
    """Host-only canonical numbering (no GPU needed): (counts[4], edges[N_e,2], faces[N_f,3])."""
    L = lib()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tv = np.ascontiguousarray(tet_vert, dtype=np.int32)
    cnt = np.zeros(4, dtype=np.int64)
    _chk(L.etpic_mesh_canonical(xyz.shape[0], _np_ptr(xyz, C.c_double), tv.shape[0], _np_ptr(tv, C.c_int32),
                                _np_ptr(cnt, C.c_int64), None, None))
    edges = np.zeros((cnt[1], 2), dtype=np.int32)
    faces = np.zeros((cnt[2], 3), dtype=np.int32)
    _chk(L.etpic_mesh_canonical(xyz.shape[0], _np_ptr(xyz, C.c_double), tv.shape[0], _np_ptr(tv, C.c_int32),
                                _np_ptr(cnt, C.c_int64), _np_ptr(edges, C.c_int32), _np_ptr(faces, C.c_int32)))
    return cnt, edges, faces


def tree_cotree(xyz, tet_vert):
    """Host-only tree-cotree split (no GPU needed): (edge_tree bool[N_e],
    face_tree bool[N_f]), True on the tree."""
    L = lib()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tv = np.ascontiguousarray(tet_vert, dtype=np.int32)
    cnt, _, _ = mesh_canonical(xyz, tv)
    et = np.zeros(int(cnt[1]), dtype=np.uint8)
    ft = np.zeros(int(cnt[2]), dtype=np.uint8)
    c4 = np.zeros(4, dtype=np.int64)
    rc = L.etpic_tree_cotree(xyz.shape[0], _np_ptr(xyz, C.c_double), tv.shape[0], _np_ptr(tv, C.c_int32),
                             _np_ptr(et, C.c_uint8), _np_ptr(ft, C.c_uint8), _np_ptr(c4, C.c_int64))
    if rc != OK:
        raise EtpicError(rc, L.etpic_qh_last_error().decode())
    assert c4[0] == et.sum() and c4[2] == ft.sum()
    return et.astype(bool), ft.astype(bool)


@dataclass
class Species:
    q: float
    m: float
    w: float = 1.0

    def c(self):
        return _Species(self.q, self.m, self.w)


def lam_to_fixed(lam):
    """float64 barycentrics [N, 3] -> the fixed-point storage of MIXED_FIXED
    (uint32 u = lam * 2^32, as int32 bits): each rounded to the nearest grid
    value in [0, 1 - 2^-32]; where the three then sum past 1 the largest gives
    up the excess (the library's own rule for the points it stores; for a
    point far outside the tet the excess is taken from the largest remaining
    coordinates in turn, none below zero)."""
    lam = np.asarray(lam, dtype=np.float64)
    u = np.clip(np.rint(lam * 4294967296.0), 0.0, 4294967295.0).astype(np.int64)
    excess = np.maximum(u.sum(axis=1) - (1 << 32), 0)
    rows = np.arange(len(u))
    for _ in range(3):
        big = np.argmax(u, axis=1)
        take = np.minimum(excess, u[rows, big])
        u[rows, big] -= take
        excess -= take
    return u.astype(np.uint32).view(np.int32)


def fixed_to_lam(u):
    """the fixed-point storage [N, 3] (int32 bits) -> float64 barycentrics (exact)"""
    return np.asarray(u).view(np.uint32).astype(np.float64) * (1.0 / 4294967296.0)


class Particles:
    """Structure-of-arrays particle state on the device (torch tensors).

    lam: float64 [3, N] (lam1, lam2, lam3), or for MIXED_FIXED int32 [3, N]
    holding the uint32 fixed-point values; vel: [3, N] float64 (FP64) or
    float32 (MIXED, MIXED_FIXED); tet: int32 [N]; ids: int64 [N] or None."""

    def __init__(self, lam, vel, tet, ids=None):
        self.lam, self.vel, self.tet, self.ids = lam, vel, tet, ids

    @property
    def n(self):
        return int(self.tet.shape[0])

    @property
    def precision(self):
        import torch
        if self.lam.dtype == torch.int32:
            return MIXED_FIXED
        return FP64 if self.vel.dtype == torch.float64 else MIXED

    @classmethod
    def from_numpy(cls, tet, lam, vel, ids=None, precision=FP64, device="cuda"):
        import torch
        vdt = torch.float64 if precision == FP64 else torch.float32
        lam_h = lam_to_fixed(lam) if precision == MIXED_FIXED else np.asarray(lam, np.float64)
        lam_t = torch.from_numpy(np.ascontiguousarray(lam_h.T)).to(device)
        vel_t = torch.from_numpy(np.ascontiguousarray(np.asarray(vel, np.float64).T)).to(device=device, dtype=vdt)
        tet_t = torch.from_numpy(np.ascontiguousarray(tet, dtype=np.int32)).to(device)
        ids_t = None if ids is None else torch.from_numpy(np.ascontiguousarray(ids, dtype=np.int64)).to(device)
        return cls(lam_t.contiguous(), vel_t.contiguous(), tet_t, ids_t)

    def empty_like(self):
        import torch
        return Particles(torch.empty_like(self.lam), torch.empty_like(self.vel), torch.empty_like(self.tet),
                         None if self.ids is None else torch.empty_like(self.ids))

    def clone(self):
        return Particles(self.lam.clone(), self.vel.clone(), self.tet.clone(),
                         None if self.ids is None else self.ids.clone())

    def to_numpy(self):
        import torch
        if self.lam.dtype == torch.int32:
            lam = fixed_to_lam(self.lam.cpu().numpy().T.copy())
        else:
            lam = self.lam.double().cpu().numpy().T.copy()
        return (self.tet.cpu().numpy(), lam, self.vel.double().cpu().numpy().T.copy(),
                None if self.ids is None else self.ids.cpu().numpy())

    def desc(self):
        """The C descriptor, after checking every array (CUDA memory, dtype,
        contiguity, [3, N] / [N] shapes, one device; EtpicError EINVAL)."""
        import torch
        n = self.n
        if self.lam.dtype == torch.int32:
            lam_dt, vel_dts = "int32", ("float32",)
        else:
            lam_dt, vel_dts = "float64", ("float64", "float32")
        _rows3(self.lam, n, "lam", lam_dt)
        vdt = str(self.vel.dtype).replace("torch.", "")
        if vdt not in vel_dts:
            raise EtpicError(EINVAL, f"vel must be {' or '.join(vel_dts)} with {lam_dt} lam, got {vdt}")
        _rows3(self.vel, n, "vel", vdt)
        _vec(self.tet, n, "tet", "int32", optional=False)
        _vec(self.ids, n, "ids", "int64")
        devs = {t.device for t in (self.lam, self.vel, self.tet, self.ids) if t is not None}
        if len(devs) != 1:
            raise EtpicError(EINVAL, f"particle arrays on several devices: {sorted(map(str, devs))}")
        d = _Particles()
        d.n = self.n
        for k in range(3):
            d.lam[k] = self.lam[k].data_ptr()
            d.vel[k] = self.vel[k].data_ptr()
        d.tet = self.tet.data_ptr()
        d.id = None if self.ids is None else self.ids.data_ptr()
        return d


class Fields:
    """Field DoFs on the device: e_env float64 [N_e, 2], b_env float64 [N_f, 2],
    optional e_dc float64 [N_e], b_dc float64 [N_f]."""

    def __init__(self, e_env, b_env, e_dc=None, b_dc=None):
        self.e_env, self.b_env, self.e_dc, self.b_dc = e_env, b_env, e_dc, b_dc

    @classmethod
    def from_numpy(cls, e_env, b_env, e_dc=None, b_dc=None, device="cuda"):
        import torch

        def cplx(z):
            z = np.asarray(z)
            return torch.from_numpy(np.ascontiguousarray(np.stack([z.real, z.imag], axis=1), dtype=np.float64)).to(device)

        def real(x):
            return None if x is None else torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(device)
        return cls(cplx(e_env), cplx(b_env), real(e_dc), real(b_dc))

    def desc(self, n_edge=None, n_face=None):
        """The C descriptor; with the mesh's edge and face counts, after
        checking every array against them (EtpicError EINVAL)."""
        if n_edge is not None:
            _vec(self.e_env, 2 * n_edge, "e_env", optional=False)
            _vec(self.e_dc, n_edge, "e_dc")
        if n_face is not None:
            _vec(self.b_env, 2 * n_face, "b_env", optional=False)
            _vec(self.b_dc, n_face, "b_dc")
        for t in (self.e_env, self.b_env, self.e_dc, self.b_dc):
            if t is not None and not t.is_contiguous():
                raise EtpicError(EINVAL, "field arrays must be contiguous")
        return _Fields(self.e_env.data_ptr(), None if self.e_dc is None else self.e_dc.data_ptr(),
                       self.b_env.data_ptr(), None if self.b_dc is None else self.b_dc.data_ptr())


def _device_buffer(nbytes, device):
    """A caller-owned device buffer for the library (uint8 torch tensor; torch's
    allocations are 512-byte aligned)."""
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=f"cuda:{device}")


class Context:
    """One etpic context bound to one HIP device.  The device buffers the
    library works in are torch tensors held here: the workspace (bound at
    creation), the mesh tables, and the solver and downshifted buffers when
    those are set up."""

    def __init__(self, device=0):
        self.device = int(device)
        self._h = C.c_void_p()
        _chk(lib().etpic_create(C.byref(self._h), self.device))
        self.counts = None
        b = C.c_size_t(0)
        _chk(lib().etpic_workspace_bytes(C.byref(b)))
        self._ws = _device_buffer(b.value, self.device)
        _chk(lib().etpic_workspace_bind(self._h, C.c_void_p(self._ws.data_ptr()), self._ws.numel()))
        self._mesh_buf = self._field_buf = self._ns_buf = self._ds_rows = None

    def close(self):
        if self._h:
            lib().etpic_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # mesh -----------------------------------------------------------------------
    def upload_mesh(self, xyz, tet_vert):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tv = np.ascontiguousarray(tet_vert, dtype=np.int32)
        cnt = np.zeros(4, dtype=np.int64)
        b = C.c_size_t(0)
        _chk(lib().etpic_mesh_sizes(xyz.shape[0], _np_ptr(xyz, C.c_double), tv.shape[0], _np_ptr(tv, C.c_int32),
                                    _np_ptr(cnt, C.c_int64), C.byref(b)))
        buf = _device_buffer(b.value, self.device)
        _chk(lib().etpic_mesh_upload(self._h, xyz.shape[0], _np_ptr(xyz, C.c_double), tv.shape[0],
                                     _np_ptr(tv, C.c_int32), C.c_void_p(buf.data_ptr()), buf.numel()))
        # the previous mesh's buffers (and those derived from it) are released
        self._mesh_buf, self._field_buf, self._ns_buf, self._ds_rows = buf, None, None, None
        _chk(lib().etpic_mesh_counts(self._h, _np_ptr(cnt, C.c_int64)))
        self.counts = tuple(int(x) for x in cnt)
        return self.counts

    @property
    def n_vert(self):
        return self.counts[0]

    @property
    def n_edge(self):
        return self.counts[1]

    @property
    def n_face(self):
        return self.counts[2]

    def _dg(self, t, name="dG", optional=True):
        return _vec(t, self.n_edge, name, optional=optional)

    def _rho(self, t, name="rho"):
        return _vec(t, self.n_vert, name)

    def _ecplx(self, t, name):
        return _vec(t, 2 * self.n_edge, name)

    def _fcplx(self, t, name):
        return _vec(t, 2 * self.n_face, name)

    @property
    def n_tet(self):
        return self.counts[3]

    def edges(self):
        out = np.zeros((self.n_edge, 2), dtype=np.int32)
        _chk(lib().etpic_mesh_edges(self._h, _np_ptr(out, C.c_int32)))
        return out

    def faces(self):
        out = np.zeros((self.n_face, 3), dtype=np.int32)
        _chk(lib().etpic_mesh_faces(self._h, _np_ptr(out, C.c_int32)))
        return out

    # particle step ----------------------------------------------------------------
    def gather_push_deposit(self, parts, species, fields, step, dt, omega, dG, rho=None, flags=STEP_XCD_REMAP,
                            stream=None):
        d = parts.desc()
        sp = species.c()
        fd = fields.desc(self.n_edge, self.n_face)
        _chk(lib().etpic_gather_push_deposit(self._h, C.byref(d), parts.precision, C.byref(sp), C.byref(fd),
                                             int(step), float(dt), float(omega), self._dg(dG), self._rho(rho),
                                             int(flags), _stream(stream)))

    def run_steps(self, parts, species, fields, step0, nsteps, dt, omega, dG, rho=None, flags=STEP_XCD_REMAP,
                  stream=None):
        """nsteps steps from step0 with fixed fields (rho after the last step)."""
        d = parts.desc()
        sp = species.c()
        fd = fields.desc(self.n_edge, self.n_face)
        _chk(lib().etpic_run_steps(self._h, C.byref(d), parts.precision, C.byref(sp), C.byref(fd), int(step0),
                                   int(nsteps), float(dt), float(omega), self._dg(dG), self._rho(rho), int(flags),
                                   _stream(stream)))

    def coarse_step(self, parts, species, snaps, t_coarse, dt_coarse, fine_steps, omega, dG, rho=None,
                    flags=STEP_XCD_REMAP, stream=None):
        """fine_steps steps from t_coarse to t_coarse + dt_coarse with the envelope
        interpolated between the three Fields snapshots (t_coarse - dt_coarse,
        t_coarse, t_coarse + dt_coarse)."""
        assert len(snaps) == 3
        d = parts.desc()
        sp = species.c()
        arr = (_Fields * 3)(*[f.desc(self.n_edge, self.n_face) for f in snaps])
        _chk(lib().etpic_coarse_step(self._h, C.byref(d), parts.precision, C.byref(sp), arr, float(t_coarse),
                                     float(dt_coarse), int(fine_steps), float(omega), self._dg(dG), self._rho(rho),
                                     int(flags), _stream(stream)))

    def sort(self, src, dst, stream=None):
        a, b = src.desc(), dst.desc()
        _chk(lib().etpic_sort(self._h, C.byref(a), C.byref(b), src.precision, _stream(stream)))

    def sort_run_steps(self, src, dst, species, fields, step0, nsteps, dt, omega, dG, rho=None,
                       flags=STEP_XCD_REMAP, stream=None):
        """sort(src, dst) then run_steps(dst, ...), the sort's scatter folded
        into the first step; the result is in dst, src is left as it was."""
        assert src.precision == dst.precision
        a, b = src.desc(), dst.desc()
        sp = species.c()
        fd = fields.desc(self.n_edge, self.n_face)
        _chk(lib().etpic_sort_run_steps(self._h, C.byref(a), C.byref(b), src.precision, C.byref(sp), C.byref(fd),
                                        int(step0), int(nsteps), float(dt), float(omega), self._dg(dG), self._rho(rho),
                                        int(flags), _stream(stream)))

    # downshifted integrator (float64) --------------------------------------------
    def ds_history(self, parts):
        """A zeroed history buffer for parts ([48, n] of the velocity type on the device)."""
        import torch
        b = C.c_size_t(0)
        _chk(lib().etpic_ds_history_bytes(int(parts.n), parts.precision, C.byref(b)))
        dt = torch.float64 if parts.precision == FP64 else torch.float32
        return torch.zeros((b.value // (dt.itemsize * max(parts.n, 1)), parts.n), dtype=dt, device="cuda")

    def ds_steps(self, parts, hist, species, fields, step0, nsteps, hist0, dt, omega, dG, rho=None,
                 flags=STEP_XCD_REMAP, stream=None):
        """nsteps downshifted steps from step0 with hist0 earlier ones in hist."""
        assert hist.is_contiguous() and hist.dtype.is_floating_point
        if self._ds_rows is None:
            b = C.c_size_t(0)
            _chk(lib().etpic_ds_rows_bytes(self._h, C.byref(b)))
            buf = _device_buffer(b.value, self.device)
            _chk(lib().etpic_ds_rows_bind(self._h, C.c_void_p(buf.data_ptr()), buf.numel()))
            self._ds_rows = buf
        d = parts.desc()
        sp = species.c()
        fd = fields.desc(self.n_edge, self.n_face)
        _chk(lib().etpic_ds_steps(self._h, C.byref(d), parts.precision, C.c_void_p(hist.data_ptr()),
                                  hist.numel() * hist.element_size(), C.byref(sp), C.byref(fd), int(step0),
                                  int(nsteps), int(hist0), float(dt), float(omega), self._dg(dG), self._rho(rho),
                                  int(flags), _stream(stream)))

    def ds_sort(self, src, dst, hist_src, hist_dst, stream=None):
        """sort(src, dst) that also moves the downshifted history."""
        assert src.precision == dst.precision
        assert hist_src.shape == hist_dst.shape and hist_src.is_contiguous() and hist_dst.is_contiguous()
        a, b = src.desc(), dst.desc()
        _chk(lib().etpic_ds_sort(self._h, C.byref(a), C.byref(b), src.precision, C.c_void_p(hist_src.data_ptr()),
                                 C.c_void_p(hist_dst.data_ptr()), hist_src.numel() * hist_src.element_size(),
                                 _stream(stream)))

    def locate(self, xyz, parts, hint=None, stream=None, raise_on_error=True):
        """Locate the points xyz (float64 [3, N] on the device) into parts.tet /
        parts.lam (parts.vel is not touched).  hint: int32 [N] start tets or None.
        Returns the status (OK, or EPARTICLE when some points were not located
        and raise_on_error is False; those get tet -1)."""
        x = _rows3(xyz, parts.n, "xyz")
        h = _vec(hint, parts.n, "hint", "int32")
        d = parts.desc()
        rc = lib().etpic_particles_locate(self._h, C.byref(d), parts.precision, x, h, _stream(stream))
        if rc != OK and (raise_on_error or rc != EPARTICLE):
            _chk(rc)
        return rc

    def positions(self, parts, xyz=None, stream=None):
        """Cartesian positions of the particles, float64 [3, N] on the device."""
        import torch
        if xyz is None:
            xyz = torch.empty((3, parts.n), dtype=torch.float64, device=parts.lam.device)
        x = _rows3(xyz, parts.n, "xyz")
        d = parts.desc()
        _chk(lib().etpic_particles_positions(self._h, C.byref(d), parts.precision, x, _stream(stream)))
        return xyz

    def vertex_charge(self, parts, species, rho, stream=None):
        d = parts.desc()
        sp = species.c()
        _chk(lib().etpic_vertex_charge(self._h, C.byref(d), parts.precision, C.byref(sp), self._rho(rho),
                                       _stream(stream)))

    def gauss_residual(self, dG, rho_new, rho_old, stream=None):
        out = np.zeros(2)
        _chk(lib().etpic_gauss_residual(self._h, self._dg(dG), self._rho(rho_new, "rho_new"),
                                        self._rho(rho_old, "rho_old"),
                                        _np_ptr(out, C.c_double), _stream(stream)))
        return float(out[0]), float(out[1])

    def last_push_slices(self):
        """slices per wavefront of the last particle-kernel launch (1 = k_push)"""
        s = C.c_int(0)
        _chk(lib().etpic_last_push_slices(self._h, C.byref(s)))
        return s.value

    def stream_probe(self, parts, flags=STEP_XCD_REMAP, stream=None):
        """the particle kernel's access pattern alone over parts (left unchanged)"""
        d = parts.desc()
        _chk(lib().etpic_stream_probe(self._h, C.byref(d), int(parts.precision), int(flags), _stream(stream)))

    def gauss_residual_noalloc(self, dG, rho_new, rho_old, stream=None):
        """gauss_residual through the allocation-free entry point."""
        out = np.zeros(2)
        _chk(lib().etpic_gauss_residual_noalloc(self._h, self._dg(dG), self._rho(rho_new, "rho_new"),
                                                self._rho(rho_old, "rho_old"),
                                                _np_ptr(out, C.c_double), _stream(stream)))
        return float(out[0]), float(out[1])

    def kernel_time(self, reset=True):
        """({"push", "coef", "walk", "push_sort"} total ms, steps) of the kernels
        of the steps run with STEP_TIMING (particle kernel only) or
        STEP_TIMING_ALL (every kernel); "push" covers the steps that update
        the particles in place, "push_sort" the sorting first steps of
        sort_run_steps, and the dict's "steps_push" / "steps_sort" count them."""
        ms = np.zeros(4)
        n = np.zeros(2, dtype=np.int64)
        _chk(lib().etpic_kernel_time(self._h, _np_ptr(ms, C.c_double), _np_ptr(n, C.c_int64), int(bool(reset))))
        return ({"push": float(ms[0]), "coef": float(ms[1]), "walk": float(ms[2]), "push_sort": float(ms[3]),
                 "steps_push": int(n[0]), "steps_sort": int(n[1])}, int(n.sum()))

    # differentiation (float64) -----------------------------------------------------
    def adjoint_workspace_bytes(self, n, nsteps, checkpoint_every):
        b = C.c_size_t(0)
        _chk(lib().etpic_adjoint_workspace(self._h, int(n), int(nsteps), int(checkpoint_every), C.byref(b)))
        return b.value

    def forward_checkpointed(self, parts, species, fields, step0, nsteps, dt, omega, checkpoint_every, workspace,
                             dG=None, stream=None):
        d = parts.desc()
        sp = species.c()
        fd = fields.desc(self.n_edge, self.n_face)
        _chk(lib().etpic_forward_checkpointed(self._h, C.byref(d), C.byref(sp), C.byref(fd), int(step0), int(nsteps),
                                              float(dt), float(omega), int(checkpoint_every),
                                              C.c_void_p(workspace.data_ptr()), workspace.numel(), self._dg(dG),
                                              _stream(stream)))

    def backward(self, n, species, fields, step0, nsteps, dt, omega, checkpoint_every, workspace, vbar, xbar,
                 grad_e, stream=None):
        """vbar, xbar: float64 [3, n] (in: final adjoints, out: initial); grad_e float64 [N_e, 2] accumulates."""
        vb = _rows3(vbar, int(n), "vbar")
        xb = _rows3(xbar, int(n), "xbar")
        ge = _vec(grad_e, 2 * self.n_edge, "grad_e")
        sp = species.c()
        fd = fields.desc(self.n_edge, self.n_face)
        _chk(lib().etpic_backward(self._h, int(n), C.byref(sp), C.byref(fd), int(step0), int(nsteps), float(dt),
                                  float(omega), int(checkpoint_every), C.c_void_p(workspace.data_ptr()),
                                  workspace.numel(), vb, xb, ge, _stream(stream)))

    # field update (side path) -------------------------------------------------------
    def field_setup(self, dt, omega, eps, mu):
        b = C.c_size_t(0)
        _chk(lib().etpic_field_bytes(self._h, float(eps), float(mu), C.byref(b)))
        buf = _device_buffer(b.value, self.device)
        _chk(lib().etpic_field_setup(self._h, float(dt), float(omega), float(eps), float(mu),
                                     C.c_void_p(buf.data_ptr()), buf.numel()))
        self._field_buf = buf
        n = C.c_int64(0)
        _chk(lib().etpic_field_nnz(self._h, C.byref(n)))
        return n.value

    def field_spmv(self, x, y, alpha, beta, stream=None):
        """y = alpha M x + beta K x; x, y float64 [N_e, 2] (complex)."""
        _chk(lib().etpic_field_spmv(self._h, self._ecplx(x, "x"), self._ecplx(y, "y"), float(np.real(alpha)),
                                    float(np.imag(alpha)),
                                    float(beta), _stream(stream)))

    def field_step(self, t_next, u, v, a, b, gdd=None, tol=1e-12, max_iter=500, stream=None, raise_on_error=True):
        """One Newmark step in place on u, v, a (float64 [N_e, 2]) and b (float64 [N_f, 2]);
        returns (status, iterations, relative residual)."""
        it = C.c_int(0)
        res = C.c_double(0.0)
        rc = lib().etpic_field_step(self._h, float(t_next), self._ecplx(u, "u"), self._ecplx(v, "v"),
                                    self._ecplx(a, "a"), self._fcplx(b, "b"), self._dg(gdd, "gdd"),
                                    float(tol), int(max_iter), C.byref(it), C.byref(res), _stream(stream))
        if raise_on_error:
            _chk(rc)
        return rc, it.value, res.value

    def ns_setup(self, eps):
        """Assemble the nodal operator of the non-solenoidal solve; returns
        (stored entries, grounded wall nodes)."""
        b = C.c_size_t(0)
        _chk(lib().etpic_ns_bytes(self._h, float(eps), C.byref(b)))
        buf = _device_buffer(b.value, self.device)
        _chk(lib().etpic_ns_setup(self._h, float(eps), C.c_void_p(buf.data_ptr()), buf.numel()))
        self._ns_buf = buf
        nnz, wall = C.c_int64(0), C.c_int64(0)
        _chk(lib().etpic_ns_info(self._h, C.byref(nnz), C.byref(wall)))
        return nnz.value, wall.value

    def ns_solve(self, G=None, rho0=None, t=0.0, omega=0.0, x_out=None, e_out=None, tol=1e-12, max_iter=2000,
                 warm=False, stream=None, raise_on_error=True):
        """Gauss-law solve: x_out float64 [N_n, 2] and e_out float64 [N_e, 2]
        (complex; either may be None); G float64 [N_e], rho0 float64 [N_n] or
        None.  Returns (status, iterations, relative residual)."""
        it = C.c_int(0)
        res = C.c_double(0.0)
        rc = lib().etpic_ns_solve(self._h, self._dg(G, "G"), self._rho(rho0, "rho0"), float(t), float(omega),
                                  _vec(x_out, 2 * self.n_vert, "x_out"), self._ecplx(e_out, "e_out"),
                                  float(tol), int(max_iter), NS_WARM if warm else 0, C.byref(it), C.byref(res),
                                  _stream(stream))
        if raise_on_error:
            _chk(rc)
        return rc, it.value, res.value

    def ns_run_steps(self, parts, species, step0, nsteps, dt, omega, G, e_work, rho0=None, ext=None, tol=1e-12,
                     max_iter=2000, flags=STEP_XCD_REMAP, warm=False, steps_per_solve=1, stream=None):
        """nsteps particle steps in the field of the charge (rho0 + D^T G),
        solved every steps_per_solve steps and held in between, plus the
        external fields ext (a Fields or None); G float64 [N_e] accumulates;
        e_work float64 [N_e] receives the field's real edge DoFs (+ ext.e_dc).
        Returns the CG iterations summed over the solves."""
        d = parts.desc()
        sp = species.c()
        fd = None if ext is None else ext.desc(self.n_edge, self.n_face)
        it = C.c_int(0)
        rc = lib().etpic_ns_run_steps(self._h, C.byref(d), parts.precision, C.byref(sp),
                                      None if fd is None else C.byref(fd), int(step0), int(nsteps),
                                      int(steps_per_solve), float(dt), float(omega), self._dg(G, "G"),
                                      self._rho(rho0, "rho0"), self._dg(e_work, "e_work"), float(tol), int(max_iter), int(flags) | (NS_WARM if warm else 0),
                                      C.byref(it), _stream(stream))
        _chk(rc)
        return it.value

    def ns_correct(self, u, e_out, G=None, rho0=None, t=0.0, omega=0.0, tol=1e-12, max_iter=2000, warm=False,
                   stream=None, raise_on_error=True):
        """e_out = u + D y with Gauss' law exact for e_out (u, e_out float64
        [N_e, 2] complex); returns (status, iterations, residual)."""
        it, res = C.c_int(0), C.c_double(0.0)
        rc = lib().etpic_ns_correct(self._h, self._dg(G, "G"), self._rho(rho0, "rho0"), float(t), float(omega),
                                    self._ecplx(u, "u"), self._ecplx(e_out, "e_out"),
                                    float(tol), int(max_iter), NS_WARM if warm else 0, C.byref(it), C.byref(res),
                                    _stream(stream))
        if raise_on_error:
            _chk(rc)
        return rc, it.value, res.value

    def sol_source(self, gdd, gs_out, tol=1e-12, max_iter=2000, warm=False, stream=None, raise_on_error=True):
        """gs_out = the field step's source gdd with its gradient part removed
        in the [*eps] inner product (float64 [N_e] device tensors; gs_out may be
        gdd); returns (status, iterations, residual)."""
        it, res = C.c_int(0), C.c_double(0.0)
        rc = lib().etpic_sol_source(self._h, self._dg(gdd, "gdd"), self._dg(gs_out, "gs_out"), float(tol),
                                    int(max_iter),
                                    NS_WARM if warm else 0, C.byref(it), C.byref(res), _stream(stream))
        if raise_on_error:
            _chk(rc)
        return rc, it.value, res.value

    def em_steps(self, parts, species, step0, nsteps, u, v, a, b, e, G, G_hist, rho0=None, tol=1e-12,
                 max_iter=2000, flags=STEP_XCD_REMAP, warm=False, split=False, stream=None):
        """nsteps steps of the electromagnetic loop (particles, field step,
        Gauss correction; split: field step on the solenoidal part plus the
        field of eq. ns_equation), all state float64 device tensors updated in
        place; returns the solver iterations summed."""
        d = parts.desc()
        sp = species.c()
        it = C.c_int(0)
        fl = int(flags) | (NS_WARM if warm else 0) | (EM_SPLIT if split else 0)
        _chk(lib().etpic_em_steps(self._h, C.byref(d), parts.precision, C.byref(sp), int(step0), int(nsteps),
                                  self._ecplx(u, "u"), self._ecplx(v, "v"), self._ecplx(a, "a"),
                                  self._fcplx(b, "b"), self._ecplx(e, "e"), self._dg(G, "G"),
                                  _vec(G_hist, 2 * self.n_edge, "G_hist"), self._rho(rho0, "rho0"), float(tol),
                                  int(max_iter), fl, C.byref(it), _stream(stream)))
        return it.value

    # checkpoint / resume of the particle state --------------------------------
    def checkpoint_write(self, parts, step, path, stream=None):
        """Saves parts (and the step index) to the host file `path`."""
        d = parts.desc()
        _chk(lib().etpic_checkpoint_write(self._h, C.byref(d), parts.precision, int(step), os.fsencode(path),
                                          _stream(stream)))

    def checkpoint_read(self, parts, path, stream=None):
        """Reads the checkpoint `path` into parts (same count, precision and id
        presence); returns its step index."""
        d = parts.desc()
        step = C.c_int64(0)
        _chk(lib().etpic_checkpoint_read(self._h, C.byref(d), parts.precision, os.fsencode(path), C.byref(step),
                                         _stream(stream)))
        return int(step.value)

    def checkpoint_load(self, path, device="cuda", stream=None):
        """(Particles, step) of the checkpoint `path`, in new device arrays."""
        import torch
        info = checkpoint_info(path)
        n, prec = info["n"], info["precision"]
        lam = torch.empty((3, n), dtype=torch.int32 if prec == MIXED_FIXED else torch.float64, device=device)
        vel = torch.empty((3, n), dtype=torch.float64 if prec == FP64 else torch.float32, device=device)
        tet = torch.empty(n, dtype=torch.int32, device=device)
        ids = torch.empty(n, dtype=torch.int64, device=device) if info["has_id"] else None
        parts = Particles(lam, vel, tet, ids)
        return parts, self.checkpoint_read(parts, path, stream=stream)

    def check(self, stream=None, raise_on_error=True):
        word = C.c_uint32(0)
        rc = lib().etpic_check(self._h, _stream(stream), C.byref(word))
        if raise_on_error:
            _chk(rc)
        return rc, int(word.value)


def _qchk(rc):
    if rc != OK:
        raise EtpicError(rc, lib().etpic_qh_last_error().decode())
    return rc


class CotreeSystem:
    """The solenoidal system of eq. sol_disc on the cotree unknowns (blocks as
    App. A prints them), on the mesh of the QhProjectors `qh`, in a device
    buffer held here.  Vectors are float64 [N, 2] (complex) device tensors:
    N_ec cotree edges, N_fc cotree faces, N_z nodes off the wall, N_f faces."""

    def __init__(self, qh, xyz, tet_vert, mu):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tv = np.ascontiguousarray(tet_vert, dtype=np.int32)
        self.qh = qh
        self._h = C.c_void_p()
        _qchk(lib().etpic_cotree_create(C.byref(self._h), qh._h, xyz.shape[0], _np_ptr(xyz, C.c_double), tv.shape[0],
                                        _np_ptr(tv, C.c_int32), float(mu)))
        b = C.c_size_t(0)
        _qchk(lib().etpic_cotree_bytes(self._h, C.byref(b)))
        self._buf = _device_buffer(b.value, qh._buf.device.index or 0)
        _qchk(lib().etpic_cotree_bind(self._h, C.c_void_p(self._buf.data_ptr()), self._buf.numel()))
        cnt = (C.c_int64 * 4)()
        _qchk(lib().etpic_cotree_counts(self._h, cnt))
        self.n_cotree_edge, self.n_cotree_face, self.n_inner_node, self.face_nnz = (int(v) for v in cnt)

    def close(self):
        if self._h:
            lib().etpic_cotree_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dims(self, block):
        """(input, output) lengths of block, or None for a number that is not a block"""
        e, f, z = self.n_cotree_edge, self.n_cotree_face, self.n_inner_node
        return {11: (f, f), 12: (e, f), 13: (z, f), 21: (e, e), 22: (f, e), 23: (z, e)}.get(int(block))

    def apply(self, block, x, y, tol=1e-13, max_iter=20000, stream=None):
        """y = Z_block x, block in 11, 12, 13, 21, 22, 23."""
        dims = self._dims(block)
        if dims is None:   # the library reports the bad block number
            xp, yp = _dptr(x), _dptr(y)
        else:
            xp, yp = _vec(x, 2 * dims[0], "x", optional=False), _vec(y, 2 * dims[1], "y", optional=False)
        _qchk(lib().etpic_cotree_apply(self._h, self.qh._h, int(block), xp, yp, float(tol),
                                       int(max_iter), _stream(stream)))

    def b_field(self, bs, b_out, tol=1e-13, max_iter=20000, stream=None):
        """b_out = P^Lambda_b C_b bs."""
        _qchk(lib().etpic_cotree_b_field(self._h, self.qh._h, _vec(bs, 2 * self.n_cotree_face, "bs"),
                                         _vec(b_out, 2 * self.qh.n_face, "b_out"), float(tol), int(max_iter),
                                         _stream(stream)))

    def step(self, dt, omega, b, es, src=None, tol=1e-11, max_iter=5000, inner_tol=1e-13, inner_max=20000,
             stream=None, raise_on_error=True):
        """One trapezoidal step of eq. sol_disc on (b, es) in place;
        returns (status, GMRES iterations, relative residual)."""
        it, res = C.c_int(0), C.c_double(0.0)
        ne = 2 * self.n_cotree_edge
        rc = lib().etpic_cotree_step(self._h, self.qh._h, float(dt), float(omega),
                                     _vec(b, 2 * self.qh.n_face, "b"), _vec(es, ne, "es"), _vec(src, ne, "src"),
                                     float(tol), int(max_iter), float(inner_tol), int(inner_max), C.byref(it),
                                     C.byref(res), _stream(stream))
        if raise_on_error:
            _qchk(rc)
        return rc, it.value, res.value


class QhProjectors:
    """Quasi-Helmholtz projectors on one mesh (its own copy of the mesh tables;
    same canonical numbering as Context.upload_mesh), in a device buffer held
    here.  Vectors are float64 [N, 2] (complex) device tensors."""

    def __init__(self, xyz, tet_vert, eps, device=0):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tv = np.ascontiguousarray(tet_vert, dtype=np.int32)
        self._h = C.c_void_p()
        _qchk(lib().etpic_qh_create(C.byref(self._h), int(device), xyz.shape[0], _np_ptr(xyz, C.c_double),
                                    tv.shape[0], _np_ptr(tv, C.c_int32), float(eps)))
        b = C.c_size_t(0)
        _qchk(lib().etpic_qh_bytes(self._h, C.byref(b)))
        self._buf = _device_buffer(b.value, int(device))
        _qchk(lib().etpic_qh_bind(self._h, C.c_void_p(self._buf.data_ptr()), self._buf.numel()))
        cnt = (C.c_int64 * 5)()
        _qchk(lib().etpic_qh_counts(self._h, cnt))
        self.n_vert, self.n_edge, self.n_face, self.n_tet, self.nnz = (int(v) for v in cnt)

    def close(self):
        if self._h:
            lib().etpic_qh_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def project_b(self, b, b_out, tol=1e-12, max_iter=5000, stream=None, raise_on_error=True):
        """b_out = P^Lambda_b b; returns (status, iterations, relative residual)."""
        it, res = C.c_int(0), C.c_double(0.0)
        nf = 2 * self.n_face
        rc = lib().etpic_qh_project_b(self._h, _vec(b, nf, "b"), _vec(b_out, nf, "b_out"), float(tol), int(max_iter),
                                      C.byref(it), C.byref(res), _stream(stream))
        if raise_on_error:
            _qchk(rc)
        return rc, it.value, res.value

    def project_e(self, d, d_sigma=None, d_lambda=None, e_ns=None, tol=1e-12, max_iter=5000, stream=None,
                  raise_on_error=True):
        """d_sigma = P^Sigma_e d, d_lambda = P^Lambda_e d, e_ns = (Sigma^T Sigma)^+ Sigma^T d;
        returns (status, iterations, relative residual)."""
        it, res = C.c_int(0), C.c_double(0.0)
        ne = 2 * self.n_edge
        rc = lib().etpic_qh_project_e(self._h, _vec(d, ne, "d"), _vec(d_sigma, ne, "d_sigma"),
                                      _vec(d_lambda, ne, "d_lambda"), _vec(e_ns, 2 * self.n_vert, "e_ns"), float(tol),
                                      int(max_iter), C.byref(it), C.byref(res), _stream(stream))
        if raise_on_error:
            _qchk(rc)
        return rc, it.value, res.value
