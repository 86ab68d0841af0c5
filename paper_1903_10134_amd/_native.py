"""ctypes binding of ``libmdpd.so`` (the C ABI in ``include/mdpd.h``).

Argument marshalling only: every step of the timestep runs in the library's
HIP kernels.  Host arrays are numpy; device arrays are torch CUDA tensors
(their ``data_ptr`` is passed with MDPD_MEM_DEVICE).  If the library is not
built this module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdpd.so")

MAX_TYPES = 8
MEM_HOST, MEM_DEVICE = 0, 1
FP64, FP32_FORCES = 0, 1
WALL_OFF, WALL_BVF = 0, 1
STATUS = {0: "MDPD_OK", -1: "MDPD_E_INVALID", -2: "MDPD_E_OOM", -3: "MDPD_E_HIP",
          -4: "MDPD_E_NONFINITE", -5: "MDPD_E_STATE", -6: "MDPD_E_UNSUPPORTED"}
KERNELS = ("sort", "nlist", "density", "force", "wall", "adjoint")


class MdpdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double * 3),
        ("rc", ctypes.c_double), ("rd", ctypes.c_double), ("kT", ctypes.c_double),
        ("dt", ctypes.c_double), ("mass", ctypes.c_double),
        ("body_force", ctypes.c_double * 3),
        ("phi_c", ctypes.c_double),
        ("A", ctypes.c_double * (MAX_TYPES * MAX_TYPES)),
        ("B", ctypes.c_double * (MAX_TYPES * MAX_TYPES)),
        ("gamma", ctypes.c_double * (MAX_TYPES * MAX_TYPES)),
        ("seed", ctypes.c_uint32),
        ("ntypes", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("wall_model", ctypes.c_int32),
        ("wall_slip", ctypes.c_double),
        ("skin", ctypes.c_double),
        ("diss_ctrl", ctypes.c_double),
        ("diss_rho", ctypes.c_double),
    ]


class Observables(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("n", ctypes.c_int64), ("n_fluid", ctypes.c_int64),
        ("ncorr_last", ctypes.c_int64), ("ncorr_total", ctypes.c_int64),
        ("ke", ctypes.c_double), ("kT", ctypes.c_double), ("pressure", ctypes.c_double),
        ("virial", ctypes.c_double), ("epot", ctypes.c_double), ("mean_rho", ctypes.c_double),
        ("momentum", ctypes.c_double * 3),
    ]


_lib = None

_SIGS = {
    "mdpd_create": ([ctypes.POINTER(Params), ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                     ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int32),
    "mdpd_create_batch": ([ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                           ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int32),
    "mdpd_read_replica_observables": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p],
                                      ctypes.c_int32),
    "mdpd_step": ([ctypes.c_void_p, ctypes.c_int64], ctypes.c_int32),
    "mdpd_read_stress": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p], ctypes.c_int32),
    "mdpd_read_stress_noalloc": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_int32], ctypes.c_int32),
    "mdpd_read_observables": ([ctypes.c_void_p, ctypes.POINTER(Observables)], ctypes.c_int32),
    "mdpd_read_list_builds": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "mdpd_read_profile": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                           ctypes.c_void_p], ctypes.c_int32),
    "mdpd_get_state": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                        ctypes.c_int32], ctypes.c_int32),
    "mdpd_debug_neighbors": ([ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p],
                             ctypes.c_int32),
    "mdpd_debug_forces": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int32),
    "mdpd_set_kernel_timing": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int32),
    "mdpd_read_kernel_timing": ([ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "mdpd_set_lanes": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32], ctypes.c_int32),
    "mdpd_autotune": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p], ctypes.c_int32),
    "mdpd_set_graph": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int32),
    "mdpd_checkpoint_size": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
    "mdpd_save_checkpoint": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32],
                             ctypes.c_int32),
    "mdpd_load_checkpoint": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32],
                             ctypes.c_int32),
    "mdpd_forward_record": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                             ctypes.c_void_p], ctypes.c_int32),
    "mdpd_backward": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32], ctypes.c_int32),
    "mdpd_destroy": ([ctypes.c_void_p], None),
    "mdpd_last_error": ([], ctypes.c_char_p),
}


def lib():
    """Load libmdpd.so; raises if it is not built (no fallback path exists).

    torch is imported first when it is installed: its bundled HIP runtime has
    the same soname as the system one, so the library then binds to it and the
    process holds a single HIP runtime (torch device pointers and streams are
    valid in the library)."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != 0:
        raise MdpdError(status, lib().mdpd_last_error().decode())


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


DEFAULT_SKIN = 0.0  # neighbour-list skin in units of r_c (0: the pair list is built every step)


def make_params(box, A, B, gamma, rc=1.0, rd=0.75, kT=1.0, dt=0.01, mass=1.0, g=(0.0, 0.0, 0.0),
                seed=0, wall_model=0, phi_c=0.5, precision=FP64, wall_slip=0.0, skin=None, diss_ctrl=0.0,
                diss_rho=0.0) -> Params:
    """Parameter block; A, B, gamma are scalars or T x T tables; skin defaults
    to DEFAULT_SKIN r_c; diss_ctrl, diss_rho: the fluid-solid dissipation
    control (eta, rho_f; eta = 0 turns it off)."""
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    B = np.atleast_2d(np.asarray(B, dtype=np.float64))
    G = np.atleast_2d(np.asarray(gamma, dtype=np.float64))
    T = A.shape[0]
    p = Params()
    p.box[:] = [float(v) for v in (box if np.ndim(box) else (box, box, box))]
    p.rc, p.rd, p.kT, p.dt, p.mass = rc, rd, kT, dt, mass
    p.body_force[:] = [float(v) for v in g]
    p.phi_c = phi_c
    for name, M in (("A", A), ("B", B), ("gamma", G)):
        if M.shape != (T, T):
            raise ValueError("A, B and gamma must have the same T x T shape")
        arr = getattr(p, name)
        for a in range(T):
            for b in range(T):
                arr[a * T + b] = M[a, b]
    p.seed = int(seed) & 0xFFFFFFFF
    p.ntypes = T
    p.precision = int(precision)
    p.wall_model = int(wall_model)
    p.wall_slip = float(wall_slip)
    p.skin = float(DEFAULT_SKIN * rc if skin is None else skin)
    p.diss_ctrl = float(diss_ctrl)
    p.diss_rho = float(diss_rho)
    return p


def _inputs(pos, vel, types, frozen):
    """Contiguous inputs, their pointers and memory kind (host numpy or CUDA tensors)."""
    if _is_torch(pos):
        import torch
        n = int(pos.shape[0])
        pos = pos.to(torch.float64).contiguous()
        vel = vel.to(torch.float64).contiguous()
        types = types.to(torch.int32).contiguous()
        frozen = frozen.to(torch.uint8).contiguous()
        keep = (pos, vel, types, frozen)
        ptrs = [t.data_ptr() for t in keep]
        mem = MEM_DEVICE
    else:
        pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))
        n = int(pos.shape[0])
        vel = np.ascontiguousarray(np.asarray(vel, dtype=np.float64).reshape(n, 3))
        types = np.ascontiguousarray(np.asarray(types, dtype=np.int32).reshape(n))
        frozen = np.ascontiguousarray(np.asarray(frozen, dtype=np.uint8).reshape(n))
        keep = (pos, vel, types, frozen)
        ptrs = [a.ctypes.data for a in keep]
        mem = MEM_HOST
    return n, keep, ptrs, mem


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def mdpd_create(params: Params, pos, vel, types, frozen, stream=None):
    """Create a system; host numpy arrays or torch CUDA tensors (all on one side)."""
    n, keep, ptrs, mem = _inputs(pos, vel, types, frozen)
    h = ctypes.c_void_p()
    _check(lib().mdpd_create(ctypes.byref(params), n, *ptrs, mem, _stream(stream), ctypes.byref(h)))
    del keep
    return h.value


def mdpd_create_batch(params_list, offsets, pos, vel, types, frozen, stream=None):
    """Create a batch of replicas: params_list[r] and particles offsets[r] ..
    offsets[r+1]-1 of the concatenated arrays."""
    nrep = len(params_list)
    arr = (Params * nrep)(*params_list)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if off.shape != (nrep + 1,):
        raise ValueError("offsets must have nrep + 1 entries")
    n, keep, ptrs, mem = _inputs(pos, vel, types, frozen)
    h = ctypes.c_void_p()
    _check(lib().mdpd_create_batch(nrep, arr, off.ctypes.data, *ptrs, mem, _stream(stream), ctypes.byref(h)))
    del keep
    return h.value


def mdpd_step(h, nsteps: int) -> None:
    _check(lib().mdpd_step(h, int(nsteps)))


def _obs_dict(o) -> dict:
    d = {k: getattr(o, k) for k, _ in Observables._fields_ if k != "momentum"}
    d["momentum"] = tuple(o.momentum)
    return d


def mdpd_read_list_builds(h) -> int:
    """List builds since creation, summed over the replicas."""
    b = ctypes.c_int64(0)
    _check(lib().mdpd_read_list_builds(h, ctypes.byref(b)))
    return int(b.value)


def mdpd_read_observables(h) -> dict:
    o = Observables()
    _check(lib().mdpd_read_observables(h, ctypes.byref(o)))
    return _obs_dict(o)


def mdpd_read_stress(h, first: int = 0, count: int = 1):
    """Pressure tensor (xx, yy, zz, xy, xz, yz) per replica: shape (count, 6)."""
    out = np.zeros(6 * max(count, 1))
    _check(lib().mdpd_read_stress(h, int(first), int(count), out.ctypes.data))
    return out[:6 * count].reshape(count, 6)


def mdpd_read_stress_noalloc(h, first: int = 0, count: int = 1, out=None):
    """The pressure tensor through the entry point that allocates nothing.
    out: None (host result, shape (count, 6)) or a float64 device tensor of
    at least 6 count elements that receives the result on the system's
    stream (returned as given)."""
    if out is None:
        res = np.zeros(6 * max(count, 1))
        _check(lib().mdpd_read_stress_noalloc(h, int(first), int(count), res.ctypes.data, MEM_HOST))
        return res[:6 * count].reshape(count, 6)
    _check(lib().mdpd_read_stress_noalloc(h, int(first), int(count), ctypes.c_void_p(out.data_ptr()),
                                          MEM_DEVICE))
    return out


def mdpd_read_replica_observables(h, first: int, count: int) -> list:
    arr = (Observables * max(count, 1))()
    _check(lib().mdpd_read_replica_observables(h, int(first), int(count), arr))
    return [_obs_dict(arr[k]) for k in range(count)]


def mdpd_read_profile(h, axis: int, nbins: int, quantity: int):
    out = np.zeros(nbins)
    _check(lib().mdpd_read_profile(h, axis, nbins, quantity, out.ctypes.data))
    return out


def mdpd_get_state(h, n: int, with_rho: bool = True, device=None):
    """Positions, velocities (n x 3) and densities in input order.  With
    device = a torch device, returns CUDA tensors written by the library."""
    if device is not None:
        import torch
        pos = torch.empty((n, 3), dtype=torch.float64, device=device)
        vel = torch.empty((n, 3), dtype=torch.float64, device=device)
        rho = torch.empty((n,), dtype=torch.float64, device=device) if with_rho else None
        _check(lib().mdpd_get_state(h, pos.data_ptr(), vel.data_ptr(),
                                    rho.data_ptr() if rho is not None else None, MEM_DEVICE))
        return pos, vel, rho
    pos = np.zeros((n, 3))
    vel = np.zeros((n, 3))
    rho = np.zeros(n) if with_rho else None
    _check(lib().mdpd_get_state(h, pos.ctypes.data, vel.ctypes.data,
                                rho.ctypes.data if rho is not None else None, MEM_HOST))
    return pos, vel, rho


def mdpd_debug_neighbors(h, n: int, cutoff: float):
    cnt = np.zeros(n, dtype=np.int64)
    hs = np.zeros(n, dtype=np.uint64)
    _check(lib().mdpd_debug_neighbors(h, float(cutoff), cnt.ctypes.data, hs.ctypes.data))
    return cnt, hs


def mdpd_debug_forces(h, n: int):
    F = np.zeros((n, 3))
    _check(lib().mdpd_debug_forces(h, F.ctypes.data))
    return F


def mdpd_set_kernel_timing(h, enable: bool) -> None:
    _check(lib().mdpd_set_kernel_timing(h, 1 if enable else 0))


def mdpd_read_kernel_timing(h, kernel: int):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(lib().mdpd_read_kernel_timing(h, int(kernel), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def mdpd_set_lanes(h, pass_: int, lanes: int) -> None:
    _check(lib().mdpd_set_lanes(h, int(pass_), int(lanes)))


def mdpd_checkpoint_size(h) -> int:
    b = ctypes.c_uint64()
    _check(lib().mdpd_checkpoint_size(h, ctypes.byref(b)))
    return b.value


def mdpd_save_checkpoint(h):
    """Checkpoint of the current state as a host uint8 array."""
    buf = np.zeros(mdpd_checkpoint_size(h), dtype=np.uint8)
    _check(lib().mdpd_save_checkpoint(h, buf.ctypes.data, buf.nbytes, MEM_HOST))
    return buf


def mdpd_load_checkpoint(h, buf) -> None:
    """Replace the state with a checkpoint (host uint8 array or CUDA tensor)."""
    if _is_torch(buf):
        _check(lib().mdpd_load_checkpoint(h, buf.data_ptr(), buf.numel() * buf.element_size(),
                                          MEM_DEVICE if buf.is_cuda else MEM_HOST))
        return
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(lib().mdpd_load_checkpoint(h, buf.ctypes.data, buf.nbytes, MEM_HOST))


def mdpd_forward_record(h, nsteps: int, every: int = 10, average: bool = False, nrep: int = 1):
    """Record a trajectory of nsteps from step 0; returns the loss terms
    (mean fluid density, virial pressure, mean fluid x-velocity): shape (3,)
    for a single system, (nrep, 3) for a batch."""
    out = np.zeros(3 * nrep)
    _check(lib().mdpd_forward_record(h, int(nsteps), int(every), 1 if average else 0, out.ctypes.data))
    return out if nrep == 1 else out.reshape(nrep, 3)


def mdpd_backward(h, w, ntypes, n: int, device=None):
    """Gradient of sum_r w[r] . loss[r] of the last recording.  ntypes: the
    type count of each replica (an int for a single system).  Returns dA, dB,
    dgamma (T x T, or a list of them per replica) and dx0, dv0 (n x 3 in
    input order; CUDA tensors when device is given)."""
    tlist = [int(ntypes)] if np.ndim(ntypes) == 0 else [int(t) for t in ntypes]
    wv = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(3 * len(tlist)))
    size = sum(t * t for t in tlist)
    flat = [np.zeros(size) for _ in range(3)]
    if device is not None:
        import torch
        dx = torch.empty((n, 3), dtype=torch.float64, device=device)
        dv = torch.empty((n, 3), dtype=torch.float64, device=device)
        ptrs, kind = (dx.data_ptr(), dv.data_ptr()), MEM_DEVICE
    else:
        dx, dv = np.zeros((n, 3)), np.zeros((n, 3))
        ptrs, kind = (dx.ctypes.data, dv.ctypes.data), MEM_HOST
    _check(lib().mdpd_backward(h, wv.ctypes.data, *[t.ctypes.data for t in flat], *ptrs, kind))

    def split(v):
        out, off = [], 0
        for t in tlist:
            out.append(v[off:off + t * t].reshape(t, t))
            off += t * t
        return out[0] if np.ndim(ntypes) == 0 else out

    return {"dA": split(flat[0]), "dB": split(flat[1]), "dgamma": split(flat[2]), "dx0": dx, "dv0": dv}


def mdpd_set_graph(h, enable: bool) -> None:
    _check(lib().mdpd_set_graph(h, 1 if enable else 0))


def mdpd_autotune(h, steps: int = 5):
    """Pick the fastest lanes per particle for the density and force passes
    (state unchanged); returns the lanes of passes 0..2."""
    out = (ctypes.c_int32 * 3)()
    _check(lib().mdpd_autotune(h, int(steps), out))
    return tuple(out)


def mdpd_destroy(h) -> None:
    if h:
        lib().mdpd_destroy(h)


def mdpd_last_error() -> str:
    return lib().mdpd_last_error().decode()


class System:
    """Owning wrapper around one mdpd_system handle."""

    def __init__(self, workload=None, precision=FP64, stream=None, device_inputs=False, params=None,
                 x=None, v=None, types=None, frozen=None, skin=None):
        if workload is not None:
            params = make_params(**workload.param_kwargs(), precision=precision, skin=skin)
            x, v, types, frozen = workload.x, workload.v, workload.types, workload.frozen
        self.params = params
        self.n = int(np.asarray(x).shape[0]) if not _is_torch(x) else int(x.shape[0])
        if device_inputs and not _is_torch(x):
            import torch
            dev = torch.device("cuda")
            x = torch.as_tensor(np.asarray(x), device=dev)
            v = torch.as_tensor(np.asarray(v), device=dev)
            types = torch.as_tensor(np.asarray(types, dtype=np.int32), device=dev)
            frozen = torch.as_tensor(np.asarray(frozen, dtype=np.uint8), device=dev)
        self.h = None
        self.h = mdpd_create(params, x, v, types, frozen, stream=stream)

    def step(self, nsteps: int = 1):
        mdpd_step(self.h, nsteps)

    def list_builds(self) -> int:
        return mdpd_read_list_builds(self.h)

    def observables(self) -> dict:
        return mdpd_read_observables(self.h)

    def profile(self, axis, nbins, quantity):
        return mdpd_read_profile(self.h, axis, nbins, quantity)

    def stress(self):
        return mdpd_read_stress(self.h, 0, 1)[0]

    def state(self, with_rho=True):
        return mdpd_get_state(self.h, self.n, with_rho)

    def neighbors(self, cutoff):
        return mdpd_debug_neighbors(self.h, self.n, cutoff)

    def forces(self):
        return mdpd_debug_forces(self.h, self.n)

    def set_lanes(self, pass_, lanes):
        mdpd_set_lanes(self.h, pass_, lanes)

    def forward_record(self, nsteps, every=10, average=False):
        return mdpd_forward_record(self.h, nsteps, every, average)

    def backward(self, w, device=None):
        return mdpd_backward(self.h, w, int(self.params.ntypes), self.n, device=device)

    def autotune(self, steps=5):
        return mdpd_autotune(self.h, steps)

    def set_graph(self, enable=True):
        mdpd_set_graph(self.h, enable)

    def save_checkpoint(self):
        return mdpd_save_checkpoint(self.h)

    def load_checkpoint(self, buf):
        mdpd_load_checkpoint(self.h, buf)

    def close(self):
        if self.h:
            mdpd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owning wrapper around a batch of replicas (mdpd_create_batch)."""

    def __init__(self, workloads, precision=FP64, stream=None, device_inputs=False, skin=None):
        self.params = [make_params(**w.param_kwargs(), precision=precision, skin=skin) for w in workloads]
        self.sizes = [int(w.x.shape[0]) for w in workloads]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        x = np.concatenate([w.x for w in workloads]) if workloads else np.zeros((0, 3))
        v = np.concatenate([w.v for w in workloads]) if workloads else np.zeros((0, 3))
        t = np.concatenate([np.asarray(w.types, np.int32) for w in workloads]) if workloads else np.zeros(0)
        f = np.concatenate([np.asarray(w.frozen, np.uint8) for w in workloads]) if workloads else np.zeros(0)
        self.n = int(self.offsets[-1])
        if device_inputs:
            import torch
            dev = torch.device("cuda")
            x, v = torch.as_tensor(x, device=dev), torch.as_tensor(v, device=dev)
            t = torch.as_tensor(t.astype(np.int32), device=dev)
            f = torch.as_tensor(f.astype(np.uint8), device=dev)
        self.h = None
        self.h = mdpd_create_batch(self.params, self.offsets, x, v, t, f, stream=stream)

    @property
    def nrep(self):
        return len(self.params)

    def step(self, nsteps: int = 1):
        mdpd_step(self.h, nsteps)

    def observables(self, first=0, count=None):
        return mdpd_read_replica_observables(self.h, first, self.nrep - first if count is None else count)

    def state(self, with_rho=True):
        return mdpd_get_state(self.h, self.n, with_rho)

    def neighbors(self, cutoff):
        return mdpd_debug_neighbors(self.h, self.n, cutoff)

    def forces(self):
        return mdpd_debug_forces(self.h, self.n)

    def set_lanes(self, pass_, lanes):
        mdpd_set_lanes(self.h, pass_, lanes)

    def autotune(self, steps=5):
        return mdpd_autotune(self.h, steps)

    def set_graph(self, enable=True):
        mdpd_set_graph(self.h, enable)

    def forward_record(self, nsteps, every=10, average=False):
        return mdpd_forward_record(self.h, nsteps, every, average, nrep=self.nrep)

    def backward(self, w, device=None):
        return mdpd_backward(self.h, w, [int(p.ntypes) for p in self.params], self.n, device=device)

    def close(self):
        if self.h:
            mdpd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
