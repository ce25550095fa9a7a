"""Python binding of the C ABI in `include/sph.h` (ctypes; argument
marshalling only -- every step of the computation runs in the HIP library).

Tensors are PyTorch tensors on the GPU; the binding passes their device
pointers and the current HIP stream.  If the library has not been built the
binding raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sph.h")

SPH_OK, SPH_STALLED, SPH_NOT_CONVERGED = 0, 1, 2
SPH_E_ARG, SPH_E_OOM, SPH_E_HIP, SPH_E_OVERFLOW, SPH_E_NONFINITE = -1, -2, -3, -4, -5
SPH_F64, SPH_F32, SPH_MIXED = 0, 1, 2
SPH_WALL_DYNAMIC, SPH_WALL_DUMMY = 0, 1
SPH_AVG_ARITH, SPH_AVG_HARMONIC = 0, 1
SPH_ROBUST, SPH_STANDARD, SPH_CG = 0, 1, 2
SPH_KERNEL_WENDLAND, SPH_KERNEL_GAUSSIAN = 0, 1
SPH_OP_CACHED, SPH_OP_ONTHEFLY, SPH_OP_PAPER32 = 0, 1, 2
SPH_CONVERGED, SPH_STATE_STALLED, SPH_PROGRESSING = 0, 1, 2
SPH_MLP_NPARAM, SPH_MLP_SAMPLE = 8835, 8
SPH_NOALLOC_MAX_N = 262144

_vp = C.c_void_p


class sph_particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", _vp), ("y", _vp), ("z", _vp), ("mass", _vp),
                ("rho", _vp), ("mu", _vp), ("type", _vp)]


class sph_domain(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("periodic", C.c_int32 * 3),
                ("h", C.c_double), ("kernel", C.c_int32)]


class sph_visc_params(C.Structure):
    _fields_ = [("dt", C.c_double), ("wall", C.c_int32), ("avg", C.c_int32),
                ("jacobi", C.c_int32), ("op_mode", C.c_int32)]


class sph_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("variant", C.c_int32),
                ("floor", C.c_double), ("true_res_period", C.c_int32), ("x0_given", C.c_int32),
                ("poll_every", C.c_int32), ("force_stall_iter", C.c_int32),
                ("force_stall_comp", C.c_int32), ("profile", C.c_int32),
                ("restart_drop", C.c_double), ("warm_params", _vp), ("warm_u", _vp * 3),
                ("fp32_scalars", C.c_int32)]


class sph_step_params(C.Structure):
    _fields_ = [("g", C.c_double * 3), ("papanastasiou", C.c_int32), ("tau0", C.c_double), ("m", C.c_double),
                ("mu0", C.c_double)]


def make_step_params(g, papa=None) -> sph_step_params:
    """Body force g (3,) and papa = (tau0, m, mu0) or None (viscosity kept)."""
    sp = sph_step_params()
    for c in range(3):
        sp.g[c] = float(g[c])
    if papa is not None:
        sp.papanastasiou = 1
        sp.tau0, sp.m, sp.mu0 = (float(v) for v in papa)
    return sp


class sph_solve_report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("state", C.c_int32 * 3),
                ("stall_count", C.c_int32 * 3), ("rr", C.c_double * 3), ("bb", C.c_double * 3),
                ("tau2", C.c_double * 3), ("true_rr", C.c_double * 3),
                ("n_true_checks", C.c_int32), ("n_replaced", C.c_int32),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int32),
                ("history_len", C.c_int32), ("setup_ms", C.c_double), ("iterate_ms", C.c_double),
                ("launches", C.c_int32), ("mat_nnz", C.c_int64), ("mat_slots", C.c_int64),
                ("apply_ms", C.c_double), ("apply_launches", C.c_int32),
                ("warm_used", C.c_int32 * 3), ("warm_rr", C.c_double * 3),
                ("plain_rr", C.c_double * 3), ("warm_scale", C.c_double), ("warm_ms", C.c_double),
                ("issued_iters", C.c_int32)]


_lib = None


def header_functions() -> list:
    """Names of the functions declared in include/sph.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|sph_status)\s*(sph_\w+)\s*\(", txt, re.M)))


def load(path: str = LIB_PATH):
    """Load libsph.so and declare the C signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    # torch first: the library must bind to the HIP runtime torch has loaded,
    # not bring in a second copy that does not know torch's device state
    import torch  # noqa: F401
    L = C.CDLL(path)
    i32, i64, st = C.c_int32, C.c_int64, C.c_int
    P = C.POINTER
    L.sph_create.argtypes = [P(_vp), i32, _vp]
    L.sph_destroy.argtypes = [_vp]
    L.sph_set_stream.argtypes = [_vp, _vp]
    L.sph_last_error.argtypes = [_vp]
    L.sph_last_error.restype = C.c_char_p
    L.sph_status_str.argtypes = [st]
    L.sph_status_str.restype = C.c_char_p
    L.sph_build_neighbors.argtypes = [_vp, P(sph_particles), P(sph_domain), P(_vp)]
    L.sph_neighbors_info.argtypes = [_vp, _vp, P(i64), P(i64)]
    L.sph_neighbors_export.argtypes = [_vp, _vp, _vp, _vp, i64, P(i64)]
    L.sph_neighbors_free.argtypes = [_vp]
    L.sph_visc_apply.argtypes = [_vp, _vp, P(sph_particles), P(sph_visc_params), i32, P(_vp), P(_vp)]
    L.sph_visc_apply_noalloc.argtypes = [_vp, _vp, P(sph_particles), P(sph_visc_params), i32, P(_vp), P(_vp)]
    L.sph_visc_solve.argtypes = [_vp, _vp, P(sph_domain), P(sph_particles), P(sph_visc_params), i32,
                                 P(_vp), P(_vp), P(sph_solve_opts), P(sph_solve_report)]
    L.sph_visc_papanastasiou.argtypes = [_vp, _vp, P(sph_particles), i32, P(_vp), C.c_double, C.c_double,
                                         C.c_double, _vp, _vp]
    L.sph_semi_implicit_step.argtypes = [_vp, P(sph_domain), P(sph_particles), P(sph_visc_params), i32,
                                         P(sph_step_params), P(sph_solve_opts), P(_vp), P(_vp), _vp,
                                         P(sph_solve_report)]
    L.sph_mlp_samples.argtypes = [_vp, _vp, P(sph_particles), P(sph_visc_params), P(_vp), P(_vp),
                                  P(_vp), _vp, P(C.c_double)]
    L.sph_mlp_warmstart.argtypes = [_vp, _vp, P(sph_particles), P(sph_visc_params), i32, P(_vp),
                                    P(_vp), _vp, P(_vp), P(C.c_double)]
    L.sph_mlp_forward.argtypes = [_vp, _vp, i64, _vp, _vp]
    L.sph_mlp_grad.argtypes = [_vp, _vp, _vp, i64, _vp, _vp, P(C.c_double)]
    L.sph_mlp_train_step.argtypes = [_vp, _vp, _vp, i64, _vp, _vp, _vp, i32, C.c_double,
                                     P(C.c_double)]
    for f in ("sph_create", "sph_destroy", "sph_set_stream", "sph_build_neighbors",
              "sph_neighbors_info", "sph_neighbors_export", "sph_neighbors_free", "sph_visc_apply",
              "sph_visc_apply_noalloc",
              "sph_visc_solve", "sph_visc_papanastasiou", "sph_semi_implicit_step", "sph_mlp_samples",
              "sph_mlp_warmstart",
              "sph_mlp_forward", "sph_mlp_grad", "sph_mlp_train_step"):
        getattr(L, f).restype = st
    _lib = L
    return L


class SphError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _ptr(t) -> int:
    return int(t.data_ptr())


def _stream_handle(device: int):
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class Particles:
    """Device arrays of one particle configuration (torch tensors on cuda,
    float64 except type: uint8).  Kept alive by this object."""
    x: object
    y: object
    z: object
    mass: object
    rho: object
    mu: object
    type: object

    @property
    def n(self) -> int:
        return int(self.x.numel())

    def c(self) -> sph_particles:
        s = sph_particles()
        s.n = self.n
        s.x, s.y, s.z = _ptr(self.x), _ptr(self.y), _ptr(self.z)
        s.mass, s.rho, s.mu, s.type = _ptr(self.mass), _ptr(self.rho), _ptr(self.mu), _ptr(self.type)
        return s


def make_domain(lo, hi, periodic, h, kernel=SPH_KERNEL_WENDLAND) -> sph_domain:
    d = sph_domain()
    for a in range(3):
        d.lo[a], d.hi[a], d.periodic[a] = float(lo[a]), float(hi[a]), int(periodic[a])
    d.h = float(h)
    d.kernel = int(kernel)
    return d


def make_params(dt, wall, avg, jacobi=True, op_mode=SPH_OP_CACHED) -> sph_visc_params:
    return sph_visc_params(float(dt), int(wall), int(avg), int(bool(jacobi)), int(op_mode))


def make_opts(tol=1e-8, max_iter=10000, variant=SPH_ROBUST, floor=-1.0, true_res_period=20,
              x0_given=False, poll_every=0, force_stall=None, profile=False,
              restart_drop=-1.0, warm_params=None, warm_u=None, fp32_scalars=False) -> sph_solve_opts:
    """Solver options; warm_params / warm_u are cuda tensors (kept alive by
    the caller for the duration of the solve)."""
    fi, fc = force_stall if force_stall is not None else (-1, -1)
    o = sph_solve_opts(float(tol), int(max_iter), int(variant), float(floor),
                       int(true_res_period), int(bool(x0_given)), int(poll_every), int(fi), int(fc),
                       int(profile), float(restart_drop))
    o.fp32_scalars = int(bool(fp32_scalars))
    if warm_params is not None:
        o.warm_params = _ptr(warm_params)
        if warm_u is not None:
            for c in range(3):
                o.warm_u[c] = _ptr(warm_u[c])
    return o


class Context:
    """sph_ctx bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise SphError(SPH_E_HIP, "no HIP device visible to torch")
        self.L = load()
        self.device = device
        h = C.c_void_p()
        s = stream if stream is not None else _stream_handle(device)
        self._check(self.L.sph_create(C.byref(h), int(device), s), "sph_create", ctx=False)
        self.h = h

    def _check(self, status: int, what: str, ctx: bool = True, soft_ok: bool = False) -> int:
        if status < 0 or (status > 0 and not soft_ok):
            msg = self.L.sph_last_error(self.h).decode() if ctx else ""
            name = self.L.sph_status_str(status).decode()
            raise SphError(status, f"{what}: {name}: {msg}")
        return status

    def close(self):
        if getattr(self, "h", None):
            self.L.sph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._check(self.L.sph_set_stream(self.h, stream), "sph_set_stream")

    # --- sph_build_neighbors / sph_neighbors_* -------------------------------
    def sph_build_neighbors(self, particles: Particles, domain: sph_domain) -> "Neighbors":
        out = C.c_void_p()
        pc = particles.c()
        self._check(self.L.sph_build_neighbors(self.h, C.byref(pc), C.byref(domain), C.byref(out)),
                    "sph_build_neighbors")
        return Neighbors(self, out)

    def sph_neighbors_info(self, nb: "Neighbors"):
        n, nnz = C.c_int64(), C.c_int64()
        self._check(self.L.sph_neighbors_info(self.h, nb.h, C.byref(n), C.byref(nnz)),
                    "sph_neighbors_info")
        return n.value, nnz.value

    def sph_neighbors_export(self, nb: "Neighbors"):
        """Canonical CSR (original indices, ascending columns) as cuda tensors."""
        import torch
        n, nnz = self.sph_neighbors_info(nb)
        dev = torch.device("cuda", self.device)
        row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
        cols = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        got = C.c_int64()
        self._check(self.L.sph_neighbors_export(self.h, nb.h, _ptr(row_ptr), _ptr(cols), nnz,
                                                C.byref(got)), "sph_neighbors_export")
        return row_ptr, cols[:got.value]

    # --- sph_visc_apply -----------------------------------------------------
    def sph_visc_apply(self, nb: "Neighbors", particles: Particles, params: sph_visc_params,
                       prec: int, x: Sequence, y: Sequence):
        xs = (C.c_void_p * 3)(*[_ptr(t) for t in x])
        ys = (C.c_void_p * 3)(*[_ptr(t) for t in y])
        pc = particles.c()
        self._check(self.L.sph_visc_apply(self.h, nb.h, C.byref(pc), C.byref(params), int(prec), xs,
                                          ys), "sph_visc_apply")

    def sph_visc_apply_noalloc(self, nb: "Neighbors", particles: Particles, params: sph_visc_params,
                               prec: int, x: Sequence, y: Sequence):
        xs = (C.c_void_p * 3)(*[_ptr(t) for t in x])
        ys = (C.c_void_p * 3)(*[_ptr(t) for t in y])
        pc = particles.c()
        self._check(self.L.sph_visc_apply_noalloc(self.h, nb.h, C.byref(pc), C.byref(params), int(prec), xs,
                                                  ys), "sph_visc_apply_noalloc")

    # --- sph_visc_papanastasiou ---------------------------------------------
    def sph_visc_papanastasiou(self, nb: "Neighbors", particles: Particles, prec: int, u: Sequence,
                               tau0: float, m: float, mu0: float, mu_out, shear_out=None):
        us = (C.c_void_p * 3)(*[_ptr(t) for t in u])
        pc = particles.c()
        self._check(self.L.sph_visc_papanastasiou(self.h, nb.h, C.byref(pc), int(prec), us, float(tau0),
                                                  float(m), float(mu0), _ptr(mu_out),
                                                  None if shear_out is None else _ptr(shear_out)),
                    "sph_visc_papanastasiou")

    # --- sph_visc_solve -----------------------------------------------------
    def sph_visc_solve(self, nb: Optional["Neighbors"], domain: Optional[sph_domain],
                       particles: Particles, params: sph_visc_params, prec: int, rhs: Sequence,
                       x: Sequence, opts: sph_solve_opts, history_cap: int = 0) -> dict:
        rs = (C.c_void_p * 3)(*[_ptr(t) for t in rhs])
        xs = (C.c_void_p * 3)(*[_ptr(t) for t in x])
        rep = sph_solve_report()
        hist = (C.c_double * (3 * max(history_cap, 1)))()
        if history_cap > 0:
            rep.history = C.cast(hist, C.POINTER(C.c_double))
            rep.history_cap = int(history_cap)
        pc = particles.c()
        st = self.L.sph_visc_solve(self.h, nb.h if nb is not None else None,
                                   C.byref(domain) if domain is not None else None, C.byref(pc),
                                   C.byref(params), int(prec), rs, xs, C.byref(opts), C.byref(rep))
        self._check(st, "sph_visc_solve", soft_ok=True)
        out = dict(status=int(st), iters=rep.iters, state=list(rep.state),
                   stall_count=list(rep.stall_count), rr=list(rep.rr), bb=list(rep.bb),
                   tau2=list(rep.tau2), true_rr=list(rep.true_rr),
                   n_true_checks=rep.n_true_checks, n_replaced=rep.n_replaced,
                   setup_ms=rep.setup_ms, iterate_ms=rep.iterate_ms, launches=rep.launches,
                   history_len=rep.history_len, mat_nnz=rep.mat_nnz, mat_slots=rep.mat_slots,
                   apply_ms=rep.apply_ms, apply_launches=rep.apply_launches,
                   warm_used=list(rep.warm_used), warm_rr=list(rep.warm_rr),
                   plain_rr=list(rep.plain_rr), warm_scale=rep.warm_scale, warm_ms=rep.warm_ms,
                   issued_iters=rep.issued_iters)
        if history_cap > 0:
            out["history"] = [[hist[3 * i + c] for c in range(3)] for i in range(rep.history_len)]
        return out

    # --- sph_semi_implicit_step ---------------------------------------------
    def sph_semi_implicit_step(self, domain: sph_domain, particles: Particles, params: sph_visc_params,
                               prec: int, step: sph_step_params, opts: sph_solve_opts, pos_out: Sequence,
                               u: Sequence, mu_out) -> list:
        """One predictor/corrector step; returns the two solve reports
        (half step, full step) as dicts with iters, status and times."""
        ps = (C.c_void_p * 3)(*[_ptr(t) for t in pos_out])
        us = (C.c_void_p * 3)(*[_ptr(t) for t in u])
        reps = (sph_solve_report * 2)()
        pc = particles.c()
        st = self.L.sph_semi_implicit_step(self.h, C.byref(domain), C.byref(pc), C.byref(params), int(prec),
                                           C.byref(step), C.byref(opts), ps, us, _ptr(mu_out), reps)
        self._check(st, "sph_semi_implicit_step", soft_ok=True)
        return [dict(status=r.status, iters=r.iters, state=list(r.state), true_rr=list(r.true_rr),
                     bb=list(r.bb), setup_ms=r.setup_ms, iterate_ms=r.iterate_ms,
                     warm_used=list(r.warm_used), warm_ms=r.warm_ms) for r in reps]


    # --- learned initial guess ----------------------------------------------
    def sph_mlp_samples(self, nb: "Neighbors", particles: Particles, params: sph_visc_params,
                        u: Sequence, rhs: Sequence, target: Optional[Sequence], samples) -> float:
        """Fills samples (cuda float32, 3 n x 8) and returns U."""
        us = (C.c_void_p * 3)(*[_ptr(t) for t in u])
        bs = (C.c_void_p * 3)(*[_ptr(t) for t in rhs])
        ts = (C.c_void_p * 3)(*[_ptr(t) for t in target]) if target is not None else None
        U = C.c_double()
        pc = particles.c()
        self._check(self.L.sph_mlp_samples(self.h, nb.h, C.byref(pc), C.byref(params), us, bs, ts,
                                           _ptr(samples), C.byref(U)), "sph_mlp_samples")
        return U.value

    def sph_mlp_warmstart(self, nb: "Neighbors", particles: Particles, params: sph_visc_params,
                          prec: int, u: Sequence, rhs: Sequence, mlp_params, x0: Sequence) -> float:
        us = (C.c_void_p * 3)(*[_ptr(t) for t in u])
        bs = (C.c_void_p * 3)(*[_ptr(t) for t in rhs])
        xs = (C.c_void_p * 3)(*[_ptr(t) for t in x0])
        U = C.c_double()
        pc = particles.c()
        self._check(self.L.sph_mlp_warmstart(self.h, nb.h, C.byref(pc), C.byref(params), int(prec),
                                             us, bs, _ptr(mlp_params), xs, C.byref(U)),
                    "sph_mlp_warmstart")
        return U.value

    def sph_mlp_forward(self, samples, n: int, mlp_params, out):
        self._check(self.L.sph_mlp_forward(self.h, _ptr(samples), int(n), _ptr(mlp_params),
                                           _ptr(out)), "sph_mlp_forward")

    def sph_mlp_grad(self, samples, idx, batch: int, mlp_params, grad) -> float:
        loss = C.c_double()
        self._check(self.L.sph_mlp_grad(self.h, _ptr(samples), _ptr(idx), int(batch),
                                        _ptr(mlp_params), _ptr(grad), C.byref(loss)),
                    "sph_mlp_grad")
        return loss.value

    def sph_mlp_train_step(self, samples, idx, batch: int, mlp_params, adam_m, adam_v, step: int,
                           lr: float, want_loss: bool = True) -> Optional[float]:
        loss = C.c_double()
        self._check(self.L.sph_mlp_train_step(self.h, _ptr(samples), _ptr(idx), int(batch),
                                              _ptr(mlp_params), _ptr(adam_m), _ptr(adam_v),
                                              int(step), float(lr),
                                              C.byref(loss) if want_loss else None),
                    "sph_mlp_train_step")
        return loss.value if want_loss else None


class Neighbors:
    """Owning wrapper of an sph_nbr handle."""

    def __init__(self, ctx: Context, h: C.c_void_p):
        self.ctx = ctx
        self.h = h

    def free(self):
        if self.h:
            self.ctx.L.sph_neighbors_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def device_particles(w, device: int = 0) -> Particles:
    """Copies the particle arrays of a workload to the GPU."""
    import torch
    dev = torch.device("cuda", device)
    t = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt).contiguous().to(dev)
    return Particles(t(w.pos[:, 0]), t(w.pos[:, 1]), t(w.pos[:, 2]), t(w.mass), t(w.rho), t(w.mu),
                     t(w.ptype, torch.uint8))


def device_vec3(a, prec: int, device: int = 0):
    """(n, 3) array -> three contiguous cuda tensors of the precision."""
    import torch
    dt = torch.float32 if prec == SPH_F32 else torch.float64
    dev = torch.device("cuda", device)
    return [torch.as_tensor(a[:, c]).to(dtype=dt).contiguous().to(dev) for c in range(3)]
