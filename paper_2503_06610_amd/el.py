"""Thin ctypes binding of libel.so (the C ABI in include/el.h).

Argument marshalling only: every step of the time step runs in the library's
HIP kernels.  PyTorch provides the device buffers and the stream.  The
binding refuses to run when libel.so is missing or cannot be loaded; there is
no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libel.so")

EL_OK, EL_EINVAL, EL_EUNSTABLE, EL_EDEVICE, EL_ENAN, EL_ENOMEM = 0, -1, -2, -3, -4, -5
EL_F64, EL_F64_SHIFTED, EL_F32, EL_F32_SHIFTED = 0, 1, 2, 3
EL_PERIODIC_Z, EL_NO_COUPLING, EL_NO_RENORM_PREDICTOR, EL_ALLOW_UNSTABLE, EL_FREEZE_DIRECTOR = 1, 2, 4, 8, 16
EL_FRANK3, EL_FREE_WALLS = 128, 256
EL_FORCE_ONE_PASS, EL_FORCE_TWO_PASS = 32, 64
EL_BUF_Q, EL_BUF_VEC3, EL_BUF_SCRATCH, EL_BUF_HALO, EL_BUF_FD_HALO = 0, 1, 2, 3, 4
EL_Q_ALIGN = 64  # values per direction of q are padded to a multiple of this (include/el.h)

PRECISIONS = {"f64": EL_F64, "f64_shifted": EL_F64_SHIFTED, "f32": EL_F32, "f32_shifted": EL_F32_SHIFTED}

# Every symbol the header declares (checked by the CPU test suite).
EXPORTED = ("el_version", "el_strerror", "el_last_error", "el_buffer_bytes", "el_validate", "el_init_lattice",
            "el_init_flow", "el_step_lbm", "el_moments", "el_step_director", "el_force", "el_run",
            "el_observables", "el_tube_drift", "el_error_norms", "el_error_norms_noalloc", "el_batch_create",
            "el_batch_step", "el_batch_capture",
            "el_batch_moments", "el_batch_observables", "el_batch_sync", "el_batch_get_tuning", "el_batch_destroy",
            "el_nn_input", "el_nn_conv_forward", "el_nn_conv_backward_data", "el_nn_work_bytes",
            "el_nn_conv_backward_weight", "el_nn_mse", "el_nn_adam", "el_nn_velocity", "el_nn_target", "el_halo_pack",
            "el_halo_unpack", "el_stream_copy", "el_fd_halo_pack", "el_fd_stage")


class ElError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__(f"{what} failed with status {status}: {detail}")
        self.status = status


class el_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("precision", C.c_int32), ("fd_ratio", C.c_int32), ("flags", C.c_int32),
                ("tau", C.c_double), ("g", C.c_double * 3), ("K", C.c_double), ("q0", C.c_double),
                ("W0", C.c_double), ("alpha", C.c_double * 6), ("alpha4p", C.c_double),
                ("K11", C.c_double), ("K22", C.c_double), ("K33", C.c_double)]


class el_state(C.Structure):
    _fields_ = [("q", C.c_void_p * 2), ("n", C.c_void_p), ("n_pred", C.c_void_p), ("dndt", C.c_void_p),
                ("u", C.c_void_p), ("F", C.c_void_p), ("scratch", C.c_void_p), ("parity", C.c_int32),
                ("reserved", C.c_int32), ("step", C.c_int64), ("solid", C.c_void_p)]


EL_MAX_TUBES = 8
_XY = (C.c_double * 2) * EL_MAX_TUBES


class el_tubes(C.Structure):
    _fields_ = [("ntubes", C.c_int32), ("reserved", C.c_int32), ("seed", _XY)]


class el_obs(C.Structure):
    _fields_ = [("mass", C.c_double), ("mom", C.c_double * 3), ("mom_phys", C.c_double * 3),
                ("max_u", C.c_double), ("max_unit_dev", C.c_double), ("nonfinite", C.c_int32),
                ("ntubes", C.c_int32), ("tube_weight", C.c_double * EL_MAX_TUBES), ("tube_centroid", _XY),
                ("tube_cs", (C.c_double * 4) * EL_MAX_TUBES)]


OBS_DOUBLES = C.sizeof(el_obs) // 8


class el_drift(C.Structure):
    _fields_ = [("obs", el_obs), ("ntubes", C.c_int32), ("ncalls", C.c_int32), ("seed", _XY), ("origin", _XY),
                ("unwrapped", _XY), ("displacement", _XY), ("step0", C.c_int64), ("step", C.c_int64)]


def make_tubes(seeds) -> el_tubes:
    """el_tubes from a list of (x, y) seeds.  The count is passed as given and
    the library validates it (1..EL_MAX_TUBES); seeds beyond the struct's
    capacity are not copied."""
    t = el_tubes()
    t.ntubes = len(seeds)
    for k, (x, y) in enumerate(seeds[:EL_MAX_TUBES]):
        t.seed[k][0], t.seed[k][1] = float(x), float(y)
    return t


def obs_dict(o: el_obs) -> dict:
    """Plain-Python view of an el_obs (per-tube arrays cut to ntubes)."""
    nt = int(o.ntubes)
    return {"mass": o.mass, "mom": np.array(o.mom[:]), "mom_phys": np.array(o.mom_phys[:]),
            "max_u": o.max_u, "max_unit_dev": o.max_unit_dev, "nonfinite": int(o.nonfinite), "ntubes": nt,
            "tube_weight": np.array(o.tube_weight[:nt]),
            "tube_centroid": np.array([o.tube_centroid[k][:] for k in range(nt)]).reshape(nt, 2),
            "tube_cs": np.array([o.tube_cs[k][:] for k in range(nt)]).reshape(nt, 4)}


class el_batch_tuning(C.Structure):
    _fields_ = [("lbm_block", C.c_int32), ("lbm_blocks_per_cu", C.c_int32), ("fd_block", C.c_int32),
                ("fd_blocks_per_cu", C.c_int32), ("tuned", C.c_int32), ("reserved", C.c_int32)]

class el_nn_vol(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nzf", C.c_int32), ("nsamples", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libel.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libel.so not found at {path}: build it with paper_2503_06610_amd/build.py")
    # torch brings its own HIP runtime; loading it before this library's (ROCm's
    # libamdhip64.so.7) is the order that works: with libel.so loaded first, the
    # first kernel launch of libel.so reported "no ROCm-capable device" once
    # torch had initialised the GPU.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P, S, V = C.POINTER(el_params), C.POINTER(el_state), C.c_void_p
    sig = {
        "el_version": (C.c_int, []),
        "el_strerror": (C.c_char_p, [C.c_int]),
        "el_last_error": (C.c_char_p, []),
        "el_buffer_bytes": (C.c_size_t, [P, C.c_int32]),
        "el_validate": (C.c_int, [P]),
        "el_init_lattice": (C.c_int, [P, S, V, V]),
        "el_init_flow": (C.c_int, [P, S, V, V]),
        "el_step_lbm": (C.c_int, [P, S, C.c_int32, C.c_int32, V]),
        "el_moments": (C.c_int, [P, S, V]),
        "el_step_director": (C.c_int, [P, S, V]),
        "el_force": (C.c_int, [P, S, V]),
        "el_run": (C.c_int, [P, S, C.c_int64, V]),
        "el_observables": (C.c_int, [P, S, C.POINTER(el_tubes), V, V]),
        "el_error_norms": (C.c_int, [P, V, V, C.c_int32, V, V, V]),
        "el_error_norms_noalloc": (C.c_int, [P, V, V, C.c_int32, V, V]),
        "el_tube_drift": (C.c_int, [P, S, V, V]),
        "el_halo_pack": (C.c_int, [P, S, V, V]),
        "el_stream_copy": (C.c_int, [V, V, C.c_size_t, V]),
        "el_halo_unpack": (C.c_int, [P, S, V, V, V]),
        "el_fd_halo_pack": (C.c_int, [P, S, C.c_int32, V, V]),
        "el_fd_stage": (C.c_int, [P, S, C.c_int32, V, V, V]),
        "el_batch_create": (C.c_int, [P, S, C.c_int32, C.POINTER(el_batch_tuning), V, C.POINTER(C.c_void_p)]),
        "el_batch_step": (C.c_int, [V, C.c_int32, V]),
        "el_batch_capture": (C.c_int, [V, V]),
        "el_batch_moments": (C.c_int, [V, V]),
        "el_batch_observables": (C.c_int, [V, C.POINTER(el_tubes), V, V]),
        "el_batch_sync": (C.c_int, [V, S, C.c_int32]),
        "el_batch_get_tuning": (C.c_int, [V, C.POINTER(el_batch_tuning)]),
        "el_batch_destroy": (C.c_int, [V]),
        "el_nn_input": (C.c_int, [P, V, V, C.c_int32, C.c_int32, C.c_float, V]),
        "el_nn_conv_forward": (C.c_int, [C.POINTER(el_nn_vol), C.c_int32, C.c_int32, V, V, V, C.c_int32, V, V]),
        "el_nn_conv_backward_data": (C.c_int, [C.POINTER(el_nn_vol), C.c_int32, C.c_int32, V, V, V, V, V]),
        "el_nn_work_bytes": (C.c_size_t, [C.POINTER(el_nn_vol), C.c_int32, C.c_int32]),
        "el_nn_conv_backward_weight": (C.c_int, [C.POINTER(el_nn_vol), C.c_int32, C.c_int32, V, V, V, C.c_size_t,
                                                 V, V, V]),
        "el_nn_mse": (C.c_int, [C.POINTER(el_nn_vol), V, V, V, V, C.c_int32, V]),
        "el_nn_adam": (C.c_int, [V, V, V, V, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32,
                                 V, V, C.c_int32, C.c_int32, V]),
        "el_nn_velocity": (C.c_int, [P, V, C.c_int32, C.c_int32, C.c_float, V, V]),
        "el_nn_target": (C.c_int, [P, V, C.c_int32, C.c_int32, C.c_float, V, V]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != EL_OK:
        raise ElError(status, what, load().el_last_error().decode())


def make_params(prob, precision: str = "f32_shifted") -> el_params:
    """el_params from a seeded Problem (paper_2503_06610_amd.inputs)."""
    p = el_params()
    p.nx, p.ny, p.nz = prob.nx, prob.ny, prob.nz
    p.precision = PRECISIONS[precision]
    p.fd_ratio = int(prob.fd_ratio)
    flags = 0
    if prob.periodic_z:
        flags |= EL_PERIODIC_Z
    if not prob.coupling:
        flags |= EL_NO_COUPLING
    if not prob.renorm_predictor:
        flags |= EL_NO_RENORM_PREDICTOR
    if prob.frank3:
        flags |= EL_FRANK3
    if prob.free_walls:
        flags |= EL_FREE_WALLS
    p.flags = flags
    p.tau = float(prob.tau)
    p.g = (C.c_double * 3)(*prob.g)
    p.K, p.q0, p.W0 = float(prob.K), float(prob.q0), float(prob.W0)
    p.alpha = (C.c_double * 6)(*prob.alpha)
    p.alpha4p = float(prob.alpha4p)
    p.K11, p.K22, p.K33 = float(prob.K11), float(prob.K22), float(prob.K33)
    return p


def validate(params: el_params) -> int:
    return load().el_validate(C.byref(params))


def buffer_bytes(params: el_params, which: int) -> int:
    return int(load().el_buffer_bytes(C.byref(params), which))


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Lattice:
    """Device buffers of one channel (torch tensors) and the C-ABI calls on them."""

    def __init__(self, prob, precision: str = "f32_shifted", device: str = "cuda", allow_unstable: bool = False,
                 freeze_director: bool = False, force_kernel: str = "auto", solid=None):
        """solid: optional obstacle mask, shape (nzf, ny, nx), nonzero = solid node."""
        import torch
        self.lib = load()
        self.prob = prob
        self.precision = precision
        self.params = make_params(prob, precision)
        if allow_unstable:
            self.params.flags |= EL_ALLOW_UNSTABLE
        if freeze_director:
            self.params.flags |= EL_FREEZE_DIRECTOR
        self.params.flags |= {"auto": 0, "one_pass": EL_FORCE_ONE_PASS, "two_pass": EL_FORCE_TWO_PASS}[force_kernel]
        _check(self.lib.el_validate(C.byref(self.params)), "el_validate")
        self.dtype = torch.float64 if precision.startswith("f64") else torch.float32
        self.N = prob.fluid_nodes
        dev = torch.device(device)
        # q: 19 direction arrays of N values, each padded to qs (a multiple of EL_Q_ALIGN)
        self.qs = -(-self.N // EL_Q_ALIGN) * EL_Q_ALIGN
        self.q = [torch.empty((19, self.qs), dtype=self.dtype, device=dev) for _ in range(2)]
        mk = lambda: torch.zeros(prob.shape(3), dtype=self.dtype, device=dev)
        self.n, self.n_pred, self.dndt, self.u, self.F = mk(), mk(), mk(), mk(), mk()
        nscratch = buffer_bytes(self.params, EL_BUF_SCRATCH)
        self.scratch = torch.empty(nscratch, dtype=torch.uint8, device=dev)
        self.obs_buf = torch.zeros(OBS_DOUBLES, dtype=torch.float64, device=dev)
        assert self.q[0].numel() * self.q[0].element_size() == buffer_bytes(self.params, EL_BUF_Q)
        self.state = el_state()
        self.state.q = (C.c_void_p * 2)(self.q[0].data_ptr(), self.q[1].data_ptr())
        self.state.n = self.n.data_ptr()
        self.state.n_pred = self.n_pred.data_ptr()
        self.state.dndt = self.dndt.data_ptr()
        self.state.u = self.u.data_ptr()
        self.state.F = self.F.data_ptr()
        self.state.scratch = self.scratch.data_ptr()
        self.state.parity = 0
        self.state.step = 0
        self.solid = None
        if solid is not None:
            m = np.ascontiguousarray(np.asarray(solid) != 0, dtype=np.uint8).reshape(prob.shape(1)[1:])
            self.solid = torch.from_numpy(m).to(dev)
            self.state.solid = self.solid.data_ptr()

    # -- the C-ABI entry points ---------------------------------------------
    def init_lattice(self, n0, stream=None):
        import torch
        t = torch.as_tensor(np.ascontiguousarray(n0) if isinstance(n0, np.ndarray) else n0)
        t = t.to(device=self.n.device, dtype=self.dtype).contiguous().reshape(self.prob.shape(3))
        self._n0 = t  # keep alive until the copy kernel ran
        _check(self.lib.el_init_lattice(C.byref(self.params), C.byref(self.state), C.c_void_p(t.data_ptr()),
                                        _stream_ptr(stream)), "el_init_lattice")

    def init_flow(self, u0, stream=None):
        import torch
        t = torch.as_tensor(u0).to(device=self.n.device, dtype=self.dtype).contiguous()
        self._u0 = t
        _check(self.lib.el_init_flow(C.byref(self.params), C.byref(self.state), C.c_void_p(t.data_ptr()),
                                     _stream_ptr(stream)), "el_init_flow")

    def step_lbm(self, nsteps: int = 1, write_u: bool = True, stream=None):
        _check(self.lib.el_step_lbm(C.byref(self.params), C.byref(self.state), int(nsteps), int(bool(write_u)),
                                    _stream_ptr(stream)), "el_step_lbm")

    def moments(self, stream=None):
        _check(self.lib.el_moments(C.byref(self.params), C.byref(self.state), _stream_ptr(stream)), "el_moments")

    def step_director(self, stream=None):
        _check(self.lib.el_step_director(C.byref(self.params), C.byref(self.state), _stream_ptr(stream)),
               "el_step_director")

    def force(self, stream=None):
        _check(self.lib.el_force(C.byref(self.params), C.byref(self.state), _stream_ptr(stream)), "el_force")

    def run(self, T: int, stream=None):
        _check(self.lib.el_run(C.byref(self.params), C.byref(self.state), int(T), _stream_ptr(stream)), "el_run")

    def observables_to(self, ptr: int, seeds=None, stream=None):
        """Device-side observables into the el_obs at device address ptr; no
        host synchronisation (read it later with decode_obs)."""
        tb = C.byref(make_tubes(seeds)) if seeds is not None else None
        _check(self.lib.el_observables(C.byref(self.params), C.byref(self.state), tb, C.c_void_p(ptr),
                                       _stream_ptr(stream)), "el_observables")

    def observables(self, seeds=None, stream=None) -> dict:
        """FP64 observables; seeds: the tubes' (x, y) seeds (None: one tube)."""
        self.observables_to(self.obs_buf.data_ptr(), seeds, stream)
        raw = self.obs_buf.cpu().numpy().tobytes()
        return obs_dict(el_obs.from_buffer_copy(raw))

    def track_drift(self, seeds=None, stream=None) -> dict:
        """Advance this lattice's FP64 tube-drift tracker (el_tube_drift); the
        first call sets the tubes' seeds (default: one tube at the centre)."""
        import torch
        if not hasattr(self, "drift_buf"):
            d0 = el_drift()
            seeds = seeds if seeds is not None else [(self.prob.nx / 2.0, self.prob.ny / 2.0)]
            d0.ntubes = len(seeds)
            for k, (x, y) in enumerate(seeds[:EL_MAX_TUBES]):
                d0.seed[k][0], d0.seed[k][1] = float(x), float(y)
            host = np.frombuffer(bytes(d0) + b"\0" * (-C.sizeof(el_drift) % 8), dtype=np.float64).copy()
            self.drift_buf = torch.from_numpy(host).to(self.n.device)
        _check(self.lib.el_tube_drift(C.byref(self.params), C.byref(self.state), C.c_void_p(self.drift_buf.data_ptr()),
                                      _stream_ptr(stream)), "el_tube_drift")
        d = el_drift.from_buffer_copy(self.drift_buf.cpu().numpy().tobytes()[:C.sizeof(el_drift)])
        nt = int(d.ntubes)
        xy = lambda a: np.array([a[k][:] for k in range(nt)]).reshape(nt, 2)
        return {"centroid": xy(d.obs.tube_centroid), "unwrapped": xy(d.unwrapped), "displacement": xy(d.displacement),
                "seed": xy(d.seed), "weight": np.array(d.obs.tube_weight[:nt]), "steps": int(d.step - d.step0),
                "ncalls": d.ncalls}

    def error_norms(self, a, ref, stream=None) -> dict:
        """Error sums of a device field `a` (this lattice's dtype) against an
        FP64 reference (numpy or tensor) of the same shape."""
        import torch
        at = a.contiguous()
        if at.dtype != self.dtype:
            raise TypeError(f"error_norms: field is {at.dtype}, the lattice computes in {self.dtype}")
        ncomp = at.shape[0]
        rt = torch.as_tensor(ref, dtype=torch.float64).to(at.device).contiguous()
        out = torch.zeros(10, dtype=torch.float64, device=at.device)
        _check(self.lib.el_error_norms(C.byref(self.params), C.c_void_p(at.data_ptr()), C.c_void_p(rt.data_ptr()),
                                       int(ncomp), C.c_void_p(self.scratch.data_ptr()), C.c_void_p(out.data_ptr()),
                                       _stream_ptr(stream)), "el_error_norms")
        v = out.cpu().numpy()
        res = {"rel_l2": float(np.sqrt(v[0] / v[1])) if v[1] > 0 else float(np.sqrt(v[0])),
               "eps": float(v[2] / v[3]) if v[3] > 0 else float(v[2])}
        res["eps_comp"] = [float(v[4 + 2 * c] / v[5 + 2 * c]) if v[5 + 2 * c] > 0 else float(v[4 + 2 * c])
                           for c in range(ncomp)]
        return res

    # -- field access ----------------------------------------------------------
    @property
    def step(self) -> int:
        return int(self.state.step)

    def q_current(self):
        return self.q[self.state.parity]

    def halo_buffer(self):
        """A device buffer for el_halo_pack of this lattice."""
        import torch
        n = buffer_bytes(self.params, EL_BUF_HALO)
        return torch.empty(n, dtype=torch.uint8, device=self.n.device)

    def halo_pack(self, out, stream=None):
        _check(self.lib.el_halo_pack(C.byref(self.params), C.byref(self.state), C.c_void_p(out.data_ptr()),
                                     _stream_ptr(stream)), "el_halo_pack")

    def halo_unpack(self, lower, upper, stream=None):
        _check(self.lib.el_halo_unpack(C.byref(self.params), C.byref(self.state), C.c_void_p(lower.data_ptr()),
                                       C.c_void_p(upper.data_ptr()), _stream_ptr(stream)), "el_halo_unpack")

    def fd_halo_buffer(self):
        """A device buffer for el_fd_halo_pack of this lattice."""
        import torch
        n = buffer_bytes(self.params, EL_BUF_FD_HALO)
        return torch.empty(n, dtype=torch.uint8, device=self.n.device)

    def fd_halo_pack(self, stage: int, out, stream=None):
        _check(self.lib.el_fd_halo_pack(C.byref(self.params), C.byref(self.state), int(stage),
                                        C.c_void_p(out.data_ptr()), _stream_ptr(stream)), "el_fd_halo_pack")

    def fd_stage(self, stage: int, lower, upper, stream=None):
        _check(self.lib.el_fd_stage(C.byref(self.params), C.byref(self.state), int(stage),
                                    C.c_void_p(lower.data_ptr()), C.c_void_p(upper.data_ptr()), _stream_ptr(stream)),
               "el_fd_stage")

    def _field(self, name: str):
        if name == "q":  # the N values of each direction, without the padding
            return self.q_current()[:, :self.N].view((19,) + self.prob.shape(1)[1:])
        return {"n": self.n, "nP": self.n_pred, "u": self.u, "F": self.F}[name]

    def get(self, name: str) -> np.ndarray:
        """Host copy (float64) of a field: q ([19][nzf][ny][nx]), n, nP, u, F."""
        import torch
        torch.cuda.synchronize()
        return self._field(name).detach().to("cpu", torch.float64).numpy()

    def set(self, name: str, arr):
        """Overwrite a field from host data (tests and warm starts)."""
        import torch
        t = self._field(name)
        t.copy_(torch.as_tensor(np.ascontiguousarray(arr)).reshape(t.shape).to(t.dtype))


class Batch:
    """A batched ensemble over Lattice objects (all of one precision), through
    el_batch_*; after capture() every step is one graph launch.  The batch
    runs on its own stream (a graph cannot be captured on the null stream),
    ordered against torch's current stream on entry and exit of every call."""

    def __init__(self, lattices, tuning=None, stream=None):
        import torch
        self.lib = load()
        self.stream = torch.cuda.Stream()
        self.lattices = list(lattices)
        n = len(self.lattices)
        self._params = (el_params * n)(*[lat.params for lat in self.lattices])
        self._states = (el_state * n)(*[lat.state for lat in self.lattices])
        self.handle = C.c_void_p()
        tu = None
        if tuning is not None:
            tu = el_batch_tuning(*tuning, 0, 0)
        self._enter()
        _check(self.lib.el_batch_create(self._params, self._states, n, C.byref(tu) if tu else None,
                                        _stream_ptr(self.stream), C.byref(self.handle)), "el_batch_create")
        self._leave()
        torch.cuda.synchronize()

    def _enter(self):
        import torch
        self.stream.wait_stream(torch.cuda.current_stream())

    def _leave(self):
        import torch
        torch.cuda.current_stream().wait_stream(self.stream)

    def step(self, nsteps: int = 1):
        self._enter()
        _check(self.lib.el_batch_step(self.handle, int(nsteps), _stream_ptr(self.stream)), "el_batch_step")
        self._leave()

    def capture(self):
        self._enter()
        _check(self.lib.el_batch_capture(self.handle, _stream_ptr(self.stream)), "el_batch_capture")
        self._leave()

    def moments(self):
        self._enter()
        _check(self.lib.el_batch_moments(self.handle, _stream_ptr(self.stream)), "el_batch_moments")
        self._leave()

    def sync(self):
        """Copy the batch's parity and step counters back into the lattices."""
        n = len(self.lattices)
        _check(self.lib.el_batch_sync(self.handle, self._states, n), "el_batch_sync")
        for lat, st in zip(self.lattices, self._states):
            lat.state.parity = st.parity
            lat.state.step = st.step

    def observables(self, seeds=None):
        """Per-channel el_obs; seeds: one list of (x, y) tube seeds per channel, or None."""
        import torch
        n = len(self.lattices)
        buf = torch.zeros(n * OBS_DOUBLES, dtype=torch.float64, device=self.lattices[0].n.device)
        tubes = (el_tubes * n)(*[make_tubes(sd) for sd in seeds]) if seeds is not None else None
        self._enter()
        _check(self.lib.el_batch_observables(self.handle, tubes, C.c_void_p(buf.data_ptr()), _stream_ptr(self.stream)),
               "el_batch_observables")
        self._leave()
        raw = buf.cpu().numpy().tobytes()
        size = C.sizeof(el_obs)
        return [el_obs.from_buffer_copy(raw[i * size:(i + 1) * size]) for i in range(n)]

    def tuning(self) -> dict:
        t = el_batch_tuning()
        _check(self.lib.el_batch_get_tuning(self.handle, C.byref(t)), "el_batch_get_tuning")
        return {f: getattr(t, f) for f, _ in el_batch_tuning._fields_}

    def close(self):
        if self.handle:
            self.lib.el_batch_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
