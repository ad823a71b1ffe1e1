"""Thin Python binding of liblbm3 (include/lbm3.h): argument marshalling only.

Every step of the lattice update runs in the HIP kernels of liblbm3.so; PyTorch supplies the
device memory (the workspace and field buffers) and the stream.  There is no CPU fallback:
if the library is missing, loading it raises.

The module-level functions carry the C names; `Simulation` strings them together.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm3.so")

LBM3_OK, LBM3_EINVAL, LBM3_ENOMEM, LBM3_EHIP, LBM3_ESTATE, LBM3_ENUMERIC, LBM3_EUNSUPPORTED = range(7)
LBM3_F64, LBM3_F32, LBM3_F32_STORE_F16 = 0, 1, 2
PRECISIONS = {"f64": LBM3_F64, "f32": LBM3_F32, "f16": LBM3_F32_STORE_F16}

# Symbols declared in include/lbm3.h.
ABI_SYMBOLS = [
    "lbm3_workspace_bytes", "lbm3_create", "lbm3_step", "lbm3_fields", "lbm3_mass",
    "lbm3_state_bytes", "lbm3_get_state", "lbm3_set_state", "lbm3_kernel_times", "lbm3_autotune",
    "lbm3_query", "lbm3_last_error", "lbm3_plan_error", "lbm3_status_string", "lbm3_destroy",
    "lbm3_set_params", "lbm3_adjoint_seed", "lbm3_adjoint_step", "lbm3_adjoint_grad",
    "lbm3_loss_seed", "lbm3_mass_device",
]


class lbm3_domain(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("y_periodic", C.c_int32), ("bc_x", C.c_int32),
        ("u_in", C.c_double), ("rho_out", C.c_double),
        ("nu", C.c_double * 3), ("sigma", C.c_double * 3), ("theta_deg", C.c_double * 2),
        ("body_force", C.c_double * 2),
        ("n_circles", C.c_int32), ("reserved", C.c_int32),
        ("circles", C.POINTER(C.c_double)), ("solid", C.POINTER(C.c_uint8)),
        ("rho_init", C.POINTER(C.c_double)),
    ]


class lbm3_options(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("graph_block_steps", C.c_int32), ("beta0", C.c_double),
        ("kernel", C.c_int32), ("tile_x", C.c_int32), ("tile_y", C.c_int32),
        ("persistent_blocks", C.c_int32), ("adjoint", C.c_int32),
        ("tune_cache", C.c_char_p),
    ]


KERNELS = {"tile": 0, "strip128": 1, "strip256": 2, "tile512": 3, "auto": -1}


class Lbm3Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm3 status {code}: {msg}")
        self.code = code


_lib = None


def library() -> C.CDLL:
    """Loads liblbm3.so (built in-tree by __graft_entry__.build()); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        # torch first: its wheel carries its own HIP and HSA runtimes, and the library must bind to
        # those (the ones that own the device memory and streams passed to it).  Loaded before
        # torch, it would bring up the system runtimes, and the second pair loaded with torch then
        # finds no device.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, dp, szp = C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_size_t)
        dom_p, opt_p = C.POINTER(lbm3_domain), C.POINTER(lbm3_options)
        sig = {
            "lbm3_workspace_bytes": (i32, [dom_p, i32, opt_p, szp]),
            "lbm3_create": (i32, [dom_p, i32, opt_p, vp, C.c_size_t, vp, C.POINTER(vp)]),
            "lbm3_step": (i32, [vp, i32]),
            "lbm3_fields": (i32, [vp, i32, vp, vp, vp, i32]),
            "lbm3_mass": (i32, [vp, dp]),
            "lbm3_state_bytes": (i32, [vp, szp]),
            "lbm3_get_state": (i32, [vp, vp]),
            "lbm3_set_state": (i32, [vp, vp]),
            "lbm3_kernel_times": (i32, [vp, i32, dp, dp]),
            "lbm3_autotune": (i32, [vp, i32, C.POINTER(C.c_int32)]),
            "lbm3_query": (i32, [vp, i32, dp]),
            "lbm3_last_error": (C.c_char_p, [vp]),
            "lbm3_plan_error": (C.c_char_p, []),
            "lbm3_status_string": (C.c_char_p, [i32]),
            "lbm3_destroy": (None, [vp]),
            "lbm3_set_params": (i32, [vp, i32, dp, dp]),
            "lbm3_adjoint_seed": (i32, [vp, vp, vp]),
            "lbm3_adjoint_step": (i32, [vp, vp, vp, vp]),
            "lbm3_adjoint_grad": (i32, [vp, dp]),
            "lbm3_loss_seed": (i32, [vp, vp, vp, vp]),
            "lbm3_mass_device": (i32, [vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class DomainArgs:
    """lbm3_domain structs for a list of workloads, keeping the host arrays alive."""

    def __init__(self, workloads: Sequence):
        self.keep: List[np.ndarray] = []
        arr = (lbm3_domain * len(workloads))()
        for d, w in zip(arr, workloads):
            solid = np.ascontiguousarray(w.solid, dtype=np.uint8)
            rho = np.ascontiguousarray(w.rho_init, dtype=np.float64)
            circ = np.ascontiguousarray(np.asarray(w.circles, dtype=np.float64).reshape(-1))
            self.keep += [solid, rho, circ]
            d.nx, d.ny, d.y_periodic, d.bc_x = w.nx, w.ny, w.y_periodic, w.bc_x
            d.u_in, d.rho_out = w.u_in, w.rho_out
            for k in range(3):
                d.nu[k] = w.nu[k]
                d.sigma[k] = w.sigma[k]
            d.theta_deg[0], d.theta_deg[1] = w.theta_deg
            d.body_force[0], d.body_force[1] = w.body_force
            d.n_circles = circ.size // 3
            d.reserved = 0
            d.circles = circ.ctypes.data_as(C.POINTER(C.c_double)) if circ.size else None
            d.solid = solid.ctypes.data_as(C.POINTER(C.c_uint8))
            d.rho_init = rho.ctypes.data_as(C.POINTER(C.c_double))
        self.array = arr
        self.n = len(workloads)


def make_options(precision="f32", graph_block_steps=0, beta0=0.0, tile=None, persistent_blocks=0,
                 kernel="tile", adjoint=False, tune_cache=None):
    o = lbm3_options()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.graph_block_steps = int(graph_block_steps)
    o.beta0 = float(beta0)
    o.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    o.tile_x, o.tile_y = (0, 0) if tile is None else (int(tile[0]), int(tile[1]))
    o.persistent_blocks = int(persistent_blocks)
    o.adjoint = 1 if adjoint else 0
    o.tune_cache = os.fsencode(tune_cache) if tune_cache else None
    return o


def _check(code: int, ctx=None) -> None:
    if code != LBM3_OK:
        L = library()
        msg = (L.lbm3_last_error(ctx) if ctx else L.lbm3_plan_error()) or b""
        raise Lbm3Error(code, msg.decode() or L.lbm3_status_string(code).decode())


# ---- the C entry points, one to one ------------------------------------------------------

def lbm3_workspace_bytes(domains: DomainArgs, options: lbm3_options) -> int:
    n = C.c_size_t(0)
    _check(library().lbm3_workspace_bytes(domains.array, domains.n, C.byref(options), C.byref(n)))
    return n.value


def lbm3_create(domains: DomainArgs, options: lbm3_options, workspace_ptr: int, nbytes: int, stream_ptr: int):
    out = C.c_void_p()
    _check(library().lbm3_create(domains.array, domains.n, C.byref(options), C.c_void_p(workspace_ptr),
                                 nbytes, C.c_void_p(stream_ptr), C.byref(out)))
    return out


def lbm3_step(ctx, nsteps: int) -> None:
    _check(library().lbm3_step(ctx, int(nsteps)), ctx)


def lbm3_fields(ctx, domain: int, rho_ptr: int, u_ptr: int, force_ptr: int, dtype: int) -> None:
    _check(library().lbm3_fields(ctx, int(domain), C.c_void_p(rho_ptr), C.c_void_p(u_ptr or None),
                                 C.c_void_p(force_ptr or None), int(dtype)), ctx)


def lbm3_mass(ctx, n_domains: int) -> np.ndarray:
    out = np.zeros(3 * n_domains)
    _check(library().lbm3_mass(ctx, out.ctypes.data_as(C.POINTER(C.c_double))), ctx)
    return out.reshape(n_domains, 3)


def lbm3_mass_device(ctx, out_ptr: int) -> None:
    _check(library().lbm3_mass_device(ctx, C.c_void_p(out_ptr)), ctx)


def lbm3_state_bytes(ctx) -> int:
    n = C.c_size_t(0)
    _check(library().lbm3_state_bytes(ctx, C.byref(n)), ctx)
    return n.value


def lbm3_get_state(ctx, dst_ptr: int) -> None:
    _check(library().lbm3_get_state(ctx, C.c_void_p(dst_ptr)), ctx)


def lbm3_set_state(ctx, src_ptr: int) -> None:
    _check(library().lbm3_set_state(ctx, C.c_void_p(src_ptr)), ctx)


def lbm3_kernel_times(ctx, nsteps: int):
    """(ms per fill launch, ms per fused-step launch)."""
    a, b = C.c_double(0), C.c_double(0)
    _check(library().lbm3_kernel_times(ctx, int(nsteps), C.byref(a), C.byref(b)), ctx)
    return a.value, b.value


def lbm3_autotune(ctx, steps: int):
    t = (C.c_int32 * 3)()
    _check(library().lbm3_autotune(ctx, int(steps), t), ctx)
    return int(t[0]), int(t[1]), int(t[2])


def lbm3_query(ctx, key: int) -> float:
    v = C.c_double(0)
    _check(library().lbm3_query(ctx, int(key), C.byref(v)), ctx)
    return v.value


def lbm3_destroy(ctx) -> None:
    library().lbm3_destroy(ctx)


def lbm3_set_params(ctx, domain: int, theta_deg, sigma) -> None:
    th = (C.c_double * 2)(*[float(v) for v in theta_deg])
    sg = (C.c_double * 3)(*[float(v) for v in sigma])
    _check(library().lbm3_set_params(ctx, int(domain), th, sg), ctx)


def lbm3_adjoint_seed(ctx, grad_rho_ptr: int, lam_ptr: int) -> None:
    _check(library().lbm3_adjoint_seed(ctx, C.c_void_p(grad_rho_ptr), C.c_void_p(lam_ptr)), ctx)


def lbm3_loss_seed(ctx, target_ptr: int, lam_ptr: int, loss_ptr: int) -> None:
    _check(library().lbm3_loss_seed(ctx, C.c_void_p(target_ptr), C.c_void_p(lam_ptr), C.c_void_p(loss_ptr)), ctx)


def lbm3_adjoint_step(ctx, state_ptr: int, lam_in_ptr: int, lam_out_ptr: int) -> None:
    _check(library().lbm3_adjoint_step(ctx, C.c_void_p(state_ptr), C.c_void_p(lam_in_ptr),
                                       C.c_void_p(lam_out_ptr)), ctx)


def lbm3_adjoint_grad(ctx, n_domains: int) -> np.ndarray:
    out = np.zeros(5 * n_domains)
    _check(library().lbm3_adjoint_grad(ctx, out.ctypes.data_as(C.POINTER(C.c_double))), ctx)
    return out.reshape(n_domains, 5)


# ---- convenience wrapper --------------------------------------------------------------------

class Simulation:
    """Domains advanced together on one GPU by liblbm3."""

    def __init__(self, workloads, precision="f32", graph_block_steps=0, tile=None,
                 persistent_blocks=0, beta0=0.0, device="cuda:0", kernel="tile", adjoint=False,
                 tune_cache=None):
        import torch

        if not isinstance(workloads, (list, tuple)):
            workloads = [workloads]
        self.workloads = list(workloads)
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.device = torch.device(device)
        self.domains = DomainArgs(self.workloads)
        self.options = make_options(precision, graph_block_steps, beta0, tile, persistent_blocks, kernel,
                                    adjoint, tune_cache)
        nbytes = lbm3_workspace_bytes(self.domains, self.options)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = lbm3_create(self.domains, self.options, self.workspace.data_ptr(), nbytes,
                               self.stream.cuda_stream)
        self.n = len(self.workloads)
        # the wetting and tension parameters in force (theta13, theta23, sigma12, sigma13, sigma23)
        self.params = np.array([[*w.theta_deg, *w.sigma] for w in self.workloads], dtype=np.float64)

    @property
    def field_dtype(self):
        import torch
        return torch.float64 if self.precision == LBM3_F64 else torch.float32

    def step(self, n: int = 1) -> None:
        lbm3_step(self.ctx, n)

    def fields(self, domain: int = 0, velocity=True, force=True) -> Dict[str, "object"]:
        import torch
        w = self.workloads[domain]
        dt = self.field_dtype
        rho = torch.empty((3, w.ny, w.nx), dtype=dt, device=self.device)
        u = torch.empty((2, w.ny, w.nx), dtype=dt, device=self.device) if velocity else None
        F = torch.empty((2, w.ny, w.nx), dtype=dt, device=self.device) if force else None
        lbm3_fields(self.ctx, domain, rho.data_ptr(), u.data_ptr() if u is not None else 0,
                    F.data_ptr() if F is not None else 0,
                    LBM3_F64 if self.precision == LBM3_F64 else LBM3_F32)
        out = {"rho": rho}
        if u is not None:
            out["u"] = u
        if F is not None:
            out["force"] = F
        return out

    def mass(self) -> np.ndarray:
        return lbm3_mass(self.ctx, self.n)

    def mass_device(self, out=None):
        """The masses of mass() into a device tensor [n, 3] (FP64), asynchronously, through the
        entry point that allocates nothing."""
        import torch
        buf = torch.empty((self.n, 3), dtype=torch.float64, device=self.device) if out is None else out
        assert buf.numel() == 3 * self.n and buf.is_contiguous() and buf.dtype == torch.float64
        lbm3_mass_device(self.ctx, buf.data_ptr())
        return buf

    def get_state(self, out=None):
        import torch
        n = lbm3_state_bytes(self.ctx)
        buf = torch.empty(n, dtype=torch.uint8, device=self.device) if out is None else out
        assert buf.numel() == n and buf.is_contiguous()
        lbm3_get_state(self.ctx, buf.data_ptr())
        return buf

    def set_state(self, buf) -> None:
        assert buf.numel() == lbm3_state_bytes(self.ctx) and buf.is_contiguous()
        lbm3_set_state(self.ctx, buf.data_ptr())

    def state_bytes(self) -> int:
        return lbm3_state_bytes(self.ctx)

    def set_params(self, domain: int, theta_deg, sigma) -> None:
        lbm3_set_params(self.ctx, domain, theta_deg, sigma)
        self.params[domain] = [*theta_deg, *sigma]

    def densities(self):
        """Partial densities of every domain, flat [3][ny][nx] per domain concatenated, zero at
        solid nodes (the output the adjoint is seeded on)."""
        import torch
        parts = []
        for d, w in enumerate(self.workloads):
            rho = self.fields(d, velocity=False, force=False)["rho"]
            fluid = torch.as_tensor(np.asarray(w.solid) == 0, device=self.device)
            parts.append((rho * fluid).reshape(-1))
        return torch.cat(parts)

    def adjoint_seed(self, grad_rho, lam) -> None:
        import torch
        g = grad_rho.to(device=self.device, dtype=torch.float64).contiguous()
        assert lam.numel() == self.state_bytes() and lam.is_contiguous()
        lbm3_adjoint_seed(self.ctx, g.data_ptr(), lam.data_ptr())

    def loss_seed(self, target, lam):
        """Phase-field mismatch loss of the current state against target (flat [3][ny][nx] per
        domain, FP64) on the device; writes lambda_T into lam and returns the per-domain losses
        (device tensor [n], FP64)."""
        import torch
        t = target.to(device=self.device, dtype=torch.float64).contiguous()
        assert t.numel() == sum(3 * w.nx * w.ny for w in self.workloads)
        assert lam.numel() == self.state_bytes() and lam.is_contiguous()
        loss = torch.empty(self.n, dtype=torch.float64, device=self.device)
        lbm3_loss_seed(self.ctx, t.data_ptr(), lam.data_ptr(), loss.data_ptr())
        return loss

    def adjoint_step(self, state, lam_in, lam_out) -> None:
        n = self.state_bytes()
        assert state.numel() == n and lam_in.numel() == n and lam_out.numel() == n
        lbm3_adjoint_step(self.ctx, state.data_ptr(), lam_in.data_ptr(), lam_out.data_ptr())

    def adjoint_grad(self) -> np.ndarray:
        return lbm3_adjoint_grad(self.ctx, self.n)

    def kernel_times(self, nsteps: int):
        return lbm3_kernel_times(self.ctx, nsteps)

    def autotune(self, steps: int = 5):
        return lbm3_autotune(self.ctx, steps)

    def query(self, key: int) -> float:
        return lbm3_query(self.ctx, key)

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None:
            lbm3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
