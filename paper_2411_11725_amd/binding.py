"""ctypes binding of libnm.so: the C entry points of include/nm.h under the same
names, plus argument marshalling from torch device tensors.

Nothing here computes: every call goes to the HIP library, which must be
built (paper_2411_11725_amd/build.py).  A missing library raises at the
first call; there is no fallback.
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_int64, c_long, c_uint, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnm.so")

NM_OK, NM_EINVAL, NM_ENOMEM, NM_EHIP, NM_ENOTREADY = 0, -1, -2, -3, -4
NM_ENONFINITE, NM_ESTEPSIZE, NM_EBUDGET, NM_EUNSUPPORTED = -5, -6, -7, -8
NM_T_EXCHANGE, NM_T_DEMAG, NM_T_ANIS, NM_T_ZEEMAN, NM_T_DMI, NM_T_CUBIC, NM_T_ALL = 1, 2, 4, 8, 16, 32, 63
NM_DMI_INTERFACIAL, NM_DMI_BULK = 0, 1
NM_RK4, NM_DP45 = 1, 2
NM_BASIS_3D, NM_BASIS_FILM = 0, 1

# entry points declared in include/nm.h
EXPORTS = [
    "nm_mesh_create", "nm_mesh_destroy", "nm_mesh_info", "nm_mesh_footprint_bytes",
    "nm_mesh_set_field", "nm_mesh_tuning", "nm_demag_tensor_init", "nm_demag_tensor_init_noalloc",
    "nm_newell_octant", "nm_heff",
    "nm_demag_cell_field", "nm_llg_rhs", "nm_energy", "nm_llg_step", "nm_adjoint_step",
    "nm_adjoint_workspace_bytes", "nm_adjoint_continuous", "nm_server_create", "nm_server_destroy", "nm_serve_submit",
    "nm_serve_poll", "nm_server_clock", "nm_profile_enable",
    "nm_profile_read", "nm_last_error",
]
PROF_SLOTS = ["xfwd", "yfwd", "conv", "yinv", "xinv", "stencil", "control", "other"]


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class nm_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", c_void_p)]


class nm_mesh_desc(ctypes.Structure):
    _fields_ = [("n", c_int * 3), ("h", c_double * 3), ("gamma", c_double), ("stream", c_void_p),
                ("basis", c_int), ("alloc", nm_allocator)]


class TorchAllocator:
    """nm_allocator hooks backed by torch's caching allocator on one device
    and stream: a mesh created with it keeps its device memory in torch's
    pool (torch.cuda.memory_allocated counts it).  Keep the object alive as
    long as the meshes made with it (the binding keeps it with each mesh)."""

    def __init__(self, device=None, stream=None):
        import torch
        self.device = torch.cuda.current_device() if device is None else torch.device(device).index
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        self.live = {}

        def _alloc(nbytes, ctx):
            p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            self.live[p] = int(nbytes)
            return p

        def _free(ptr, ctx):
            if ptr in self.live:
                del self.live[ptr]
                torch.cuda.caching_allocator_delete(ptr)

        self._c = nm_allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)

    def hooks(self):
        return self._c


_mesh_allocators = {}   # mesh handle -> allocator object kept alive with the mesh


class nm_material(ctypes.Structure):
    _fields_ = [("Ms", c_void_p), ("A", c_void_p), ("alpha", c_void_p), ("Ku", c_void_p),
                ("easy", c_void_p), ("h_cell", c_void_p), ("h_uniform", c_float * 3),
                ("drive_mask", c_void_p), ("drive_amp", c_float * 3),
                ("drive_freq", c_double), ("drive_phase", c_double), ("D", c_void_p),
                ("dmi_type", c_int), ("Kc", c_void_p), ("cubic", c_void_p)]


class nm_integrator(ctypes.Structure):
    _fields_ = [("method", c_int), ("terms", c_uint), ("rtol", c_double), ("atol", c_double),
                ("dt_min", c_double), ("dt_max", c_double), ("stop_torque", c_double),
                ("log", c_void_p), ("log_capacity", c_long)]


class nm_clock(ctypes.Structure):
    _fields_ = [("t", c_double), ("dt", c_double), ("accepted", c_long), ("rejected", c_long),
                ("rhs_evals", c_long), ("max_torque", c_double)]


class nm_server_desc(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_active", c_int), ("n_streams", c_int),
                ("attempts_per_launch", c_int)]


class nm_solve_request(ctypes.Structure):
    _fields_ = [("n", c_int * 3), ("h", c_double * 3), ("gamma", c_double), ("Ms", c_void_p),
                ("A", c_void_p), ("alpha", c_void_p), ("m0", c_void_p), ("h_uniform", c_float * 3),
                ("terms", c_uint), ("rtol", c_double), ("atol", c_double), ("dt0", c_double),
                ("t_end", c_double), ("Ku", c_void_p), ("easy", c_void_p), ("h_cell", c_void_p),
                ("D", c_void_p), ("dmi_type", c_int), ("Kc", c_void_p), ("cubic", c_void_p)]


class nm_solve_result(ctypes.Structure):
    _fields_ = [("status", c_int), ("t", c_double), ("accepted", c_long), ("rejected", c_long),
                ("rhs_evals", c_long), ("t_submit", c_double), ("t_admit", c_double),
                ("t_done", c_double)]


class NMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("nm status %d: %s" % (status, msg))
        self.status = status


_lib = None


def lib():
    """Open libnm.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnm.so not built; run paper_2411_11725_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = c_void_p
        sig = {
            "nm_mesh_create": ([POINTER(nm_mesh_desc), POINTER(nm_material), POINTER(c_void_p)], c_int),
            "nm_mesh_destroy": ([P], c_int),
            "nm_mesh_info": ([P, POINTER(c_int64), POINTER(c_int64), POINTER(c_int)], c_int),
            "nm_mesh_footprint_bytes": ([POINTER(nm_mesh_desc), c_int], ctypes.c_size_t),
            "nm_mesh_set_field": ([P, P], c_int),
            "nm_mesh_tuning": ([P, c_int, POINTER(c_int), POINTER(c_int)], c_int),
            "nm_demag_tensor_init": ([P], c_int),
            "nm_demag_tensor_init_noalloc": ([P], c_int),
            "nm_newell_octant": ([POINTER(c_int), POINTER(c_double), P, P], c_int),
            "nm_heff": ([P, P, P, c_uint, c_double], c_int),
            "nm_demag_cell_field": ([P, P, P], c_int),
            "nm_llg_rhs": ([P, P, P, c_uint, c_double], c_int),
            "nm_energy": ([P, P, c_uint, c_double, POINTER(c_double)], c_int),
            "nm_llg_step": ([P, P, POINTER(nm_clock), POINTER(nm_integrator), c_double, c_long], c_int),
            "nm_adjoint_step": ([P, P, c_double, c_double, c_int, c_uint, P, c_int, P, P, P], c_int),
            "nm_adjoint_workspace_bytes": ([P, c_int], ctypes.c_size_t),
            "nm_adjoint_continuous": ([P, P, c_double, c_double, c_int, c_uint, P, P], c_int),
            "nm_server_create": ([POINTER(nm_server_desc), POINTER(c_void_p)], c_int),
            "nm_server_destroy": ([P], c_int),
            "nm_serve_submit": ([P, POINTER(nm_solve_request), POINTER(ctypes.c_uint64)], c_int),
            "nm_serve_poll": ([P, ctypes.c_uint64, POINTER(nm_solve_result), P, c_int], c_int),
            "nm_server_clock": ([], c_double),
            "nm_profile_enable": ([P, c_int], c_int),
            "nm_profile_read": ([P, POINTER(c_double), POINTER(ctypes.c_longlong)], c_int),
            "nm_last_error": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status):
    if status != NM_OK:
        raise NMError(status, lib().nm_last_error().decode())


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- entry points
def nm_mesh_create(n, h, gamma, Ms, A, alpha, Ku=None, easy=None, h_cell=None,
                   h_uniform=(0.0, 0.0, 0.0), drive_mask=None, drive_amp=(0.0, 0.0, 0.0),
                   drive_freq=0.0, drive_phase=0.0, stream=None, basis=NM_BASIS_3D, D=None,
                   dmi_type=NM_DMI_INTERFACIAL, Kc=None, cubic=None, allocator=None):
    """Create a mesh from float32 device tensors (copied by the library).
    allocator: optional TorchAllocator (or any object with hooks()) whose
    nm_allocator hooks provide the mesh's device memory."""
    desc = nm_mesh_desc((c_int * 3)(*n), (c_double * 3)(*h), float(gamma), _stream_handle(stream),
                        int(basis), allocator.hooks() if allocator is not None else nm_allocator())
    mat = nm_material(_ptr(Ms), _ptr(A), _ptr(alpha), _ptr(Ku), _ptr(easy), _ptr(h_cell),
                      (c_float * 3)(*h_uniform), _ptr(drive_mask), (c_float * 3)(*drive_amp),
                      float(drive_freq), float(drive_phase), _ptr(D), int(dmi_type), _ptr(Kc), _ptr(cubic))
    out = c_void_p()
    _check(lib().nm_mesh_create(ctypes.byref(desc), ctypes.byref(mat), ctypes.byref(out)))
    if allocator is not None:
        _mesh_allocators[out.value] = allocator
    return out


def nm_mesh_destroy(mesh):
    _check(lib().nm_mesh_destroy(mesh))
    _mesh_allocators.pop(mesh.value if isinstance(mesh, c_void_p) else mesh, None)


def nm_mesh_info(mesh):
    nn, nc, pad = c_int64(), c_int64(), (c_int * 3)()
    _check(lib().nm_mesh_info(mesh, ctypes.byref(nn), ctypes.byref(nc), pad))
    return nn.value, nc.value, tuple(pad)


def nm_mesh_tuning(mesh, y=None, z=None):
    """(y_width, z_width) of the register-FFT passes; with y or z given,
    impose it first (0 widest, 1 half, 2 quarter)."""
    yy, zz = c_int(-1 if y is None else y), c_int(-1 if z is None else z)
    _check(lib().nm_mesh_tuning(mesh, 0 if (y is None and z is None) else 1, ctypes.byref(yy), ctypes.byref(zz)))
    return yy.value, zz.value


def nm_mesh_footprint_bytes(n, h, gamma=2.211e5, integrator=NM_DP45, basis=NM_BASIS_3D):
    desc = nm_mesh_desc((c_int * 3)(*n), (c_double * 3)(*h), float(gamma), None, int(basis))
    return lib().nm_mesh_footprint_bytes(ctypes.byref(desc), integrator)


def nm_mesh_set_field(mesh, h_cell):
    _check(lib().nm_mesh_set_field(mesh, _ptr(h_cell)))


def nm_demag_tensor_init(mesh):
    _check(lib().nm_demag_tensor_init(mesh))


def nm_demag_tensor_init_noalloc(mesh):
    _check(lib().nm_demag_tensor_init_noalloc(mesh))


def nm_newell_octant(n, h, out, stream=None):
    _check(lib().nm_newell_octant((c_int * 3)(*n), (c_double * 3)(*h), _ptr(out),
                                  _stream_handle(stream)))


def nm_heff(mesh, m, h, terms=NM_T_ALL, t=0.0):
    _check(lib().nm_heff(mesh, _ptr(m), _ptr(h), terms, float(t)))


def nm_demag_cell_field(mesh, m, out):
    _check(lib().nm_demag_cell_field(mesh, _ptr(m), _ptr(out)))


def nm_llg_rhs(mesh, m, dmdt, terms=NM_T_ALL, t=0.0):
    _check(lib().nm_llg_rhs(mesh, _ptr(m), _ptr(dmdt), terms, float(t)))


def nm_energy(mesh, m, terms=NM_T_ALL, t=0.0):
    e = (c_double * 6)()
    _check(lib().nm_energy(mesh, _ptr(m), terms, float(t), e))
    return {"exchange": e[0], "demag": e[1], "anisotropy": e[2], "zeeman": e[3], "total": e[4], "dmi": e[5]}


def nm_llg_step(mesh, m, clock, method=NM_RK4, terms=NM_T_ALL, t_end=0.0, max_steps=1 << 40,
                rtol=1e-5, atol=1e-5, dt_min=1e-20, dt_max=0.0, stop_torque=0.0, log=None):
    """Advance m in place; clock is an nm_clock updated in place."""
    integ = nm_integrator(method, terms, rtol, atol, dt_min, dt_max, stop_torque, _ptr(log),
                          0 if log is None else log.numel() // 3)
    _check(lib().nm_llg_step(mesh, _ptr(m), ctypes.byref(clock), ctypes.byref(integ),
                             float(t_end), int(max_steps)))
    return clock


def nm_adjoint_continuous(mesh, m, t_end, dt, nsteps, terms, a, grad_hcell=None):
    """Backward integration of the continuous adjoint system; m and a (device
    tensors) are updated in place, grad_hcell accumulates the field-map
    gradient."""
    _check(lib().nm_adjoint_continuous(mesh, _ptr(m), float(t_end), float(dt), int(nsteps), int(terms),
                                       _ptr(a), _ptr(grad_hcell)))


def nm_adjoint_workspace_bytes(mesh, nsteps):
    return lib().nm_adjoint_workspace_bytes(mesh, int(nsteps))


def nm_adjoint_step(mesh, m0, t0, dt, nsteps, terms, lam, dl_dm=None, dl_every=1, grad_hcell=None,
                    work=None):
    """Reverse sweep over one checkpointed RK4 segment; lam (in/out) and
    grad_hcell (accumulated) are device tensors."""
    if work is None:
        import torch
        work = torch.empty(nm_adjoint_workspace_bytes(mesh, nsteps) // 4, dtype=torch.float32,
                           device=lam.device)
    _check(lib().nm_adjoint_step(mesh, _ptr(m0), float(t0), float(dt), int(nsteps), int(terms),
                                 _ptr(dl_dm), int(dl_every), _ptr(lam), _ptr(grad_hcell), _ptr(work)))
    return work


def nm_server_create(max_active=64, n_streams=4, attempts_per_launch=8, hbm_budget=0):
    desc = nm_server_desc(int(hbm_budget), int(max_active), int(n_streams), int(attempts_per_launch))
    out = c_void_p()
    _check(lib().nm_server_create(ctypes.byref(desc), ctypes.byref(out)))
    return out


def nm_server_destroy(server):
    _check(lib().nm_server_destroy(server))


def nm_serve_submit(server, p, terms=NM_T_ALL, rtol=1e-5, atol=1e-5, dt0=1e-14, t_end=0.2e-9):
    """Submit a problem dict (see synth.make_problem; host float32 arrays).
    The optional cell arrays Ku/easy, h_cell, D (with dmi_type) and
    Kc/cubic go with the request when the dict has them; a drive does not
    (the server runs no time-dependent field)."""
    import numpy as np
    if p.get("drive_mask") is not None and any(float(v) != 0.0 for v in p.get("drive_amp", (0.0,) * 3)):
        raise ValueError("nm_serve_submit: the server runs no time-dependent drive")
    keys = ("Ms", "A", "alpha", "m0", "Ku", "easy", "h_cell", "D", "Kc", "cubic")
    keep = {k: np.ascontiguousarray(p[k], dtype=np.float32) for k in keys if p.get(k) is not None}
    ptr = {k: c_void_p(a.ctypes.data) for k, a in keep.items()}
    req = nm_solve_request((c_int * 3)(*p["n"]), (c_double * 3)(*p["h"]), float(p["gamma"]),
                           ptr["Ms"], ptr["A"], ptr["alpha"], ptr["m0"],
                           (c_float * 3)(*[float(v) for v in p["h_uniform"]]), int(terms),
                           float(rtol), float(atol), float(dt0), float(t_end),
                           ptr.get("Ku"), ptr.get("easy"), ptr.get("h_cell"), ptr.get("D"),
                           NM_DMI_BULK if p.get("dmi_type", "interfacial") == "bulk" else NM_DMI_INTERFACIAL,
                           ptr.get("Kc"), ptr.get("cubic"))
    t = ctypes.c_uint64()
    _check(lib().nm_serve_submit(server, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def nm_serve_poll(server, ticket, timeout_ms=0, m_out=None):
    """Result struct, or None while the solve is still running."""
    res = nm_solve_result()
    st = lib().nm_serve_poll(server, ctypes.c_uint64(ticket), ctypes.byref(res),
                             None if m_out is None else c_void_p(m_out.ctypes.data), int(timeout_ms))
    if st == NM_ENOTREADY:
        return None
    _check(st)
    return res


def nm_server_clock():
    return lib().nm_server_clock()


def nm_profile_enable(mesh, on=True):
    _check(lib().nm_profile_enable(mesh, 1 if on else 0))


def nm_profile_read(mesh):
    """{slot: (milliseconds, launches)} accumulated since nm_profile_enable."""
    ms = (c_double * 8)()
    cnt = (ctypes.c_longlong * 8)()
    _check(lib().nm_profile_read(mesh, ms, cnt))
    return {name: (ms[i], cnt[i]) for i, name in enumerate(PROF_SLOTS)}


def nm_last_error():
    return lib().nm_last_error().decode()


# ------------------------------------------------------------ marshalling
def mesh_from_problem(p, device="cuda", stream=None, tensor=True, allocator=None):
    """Upload a problem dict (see synth.make_problem) and create its mesh
    (allocator: optional hooks for the mesh's device memory, see
    TorchAllocator)."""
    import torch

    def dev(a):
        return None if a is None else torch.as_tensor(a, dtype=torch.float32, device=device).contiguous()

    arrays = {k: dev(p.get(k)) for k in ("Ms", "A", "alpha", "Ku", "easy", "h_cell", "drive_mask", "D", "Kc",
                                         "cubic")}
    mesh = nm_mesh_create(p["n"], p["h"], p["gamma"], arrays["Ms"], arrays["A"], arrays["alpha"],
                          Ku=arrays["Ku"], easy=arrays["easy"], h_cell=arrays["h_cell"],
                          h_uniform=tuple(float(v) for v in p["h_uniform"]),
                          drive_mask=arrays["drive_mask"],
                          drive_amp=tuple(float(v) for v in p["drive_amp"]),
                          drive_freq=p["drive_freq"], drive_phase=p["drive_phase"], stream=stream,
                          basis=NM_BASIS_FILM if p.get("basis", "3d") == "film" else NM_BASIS_3D,
                          D=arrays["D"],
                          dmi_type=NM_DMI_BULK if p.get("dmi_type", "interfacial") == "bulk" else NM_DMI_INTERFACIAL,
                          Kc=arrays["Kc"], cubic=arrays["cubic"], allocator=allocator)
    if tensor:
        nm_demag_tensor_init(mesh)
    return mesh
