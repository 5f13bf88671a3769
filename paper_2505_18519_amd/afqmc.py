"""Thin Python binding of libafqmc (the C ABI in include/afqmc.h).

Argument marshalling only: every function below checks the torch tensors it
is given (device, dtype, contiguity and size, so that no kernel can be handed
a buffer smaller than its grid assumes) and passes raw device pointers and the
current HIP stream to the C function of the same name.  There is no fallback:
if the HIP library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_size_t, c_uint32, c_uint64, c_void_p

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libafqmc.so")

HIDDEN_ISING, HIDDEN_GAUSS = 0, 1
WEIGHT_SEPARATE, WEIGHT_COMBINED, WEIGHT_HALFPLANE, WEIGHT_LOCAL = 0, 1, 2, 3
PROPOSAL_PRIOR, PROPOSAL_RW, PROPOSAL_LEARNED = 0, 1, 2
PREC_FP64, PREC_FP32, PREC_BF16, PREC_BF16X3 = 0, 1, 2, 3
MLP_HIDDEN = 256
TAG_FIELD, TAG_PROPOSAL, TAG_ACCEPT, TAG_COMB, TAG_INIT = 1, 2, 3, 4, 5
INIT_STEP, MEASURE_STEP = 1 << 63, 1 << 62     # AFQMC_INIT_STEP, AFQMC_MEASURE_STEP
TRIAL_JASTROW, TRIAL_SLICES = 0, 1
NUMERIC_ELOC, NUMERIC_XBAR, NUMERIC_WEIGHT, NUMERIC_HANDOFF = 1, 2, 4, 8
E_NUMERIC = 5

STATUS = {0: "OK", 1: "E_INVALID", 2: "E_SHAPE", 3: "E_DEVICE", 4: "E_NOMEM",
          5: "E_NUMERIC", 6: "E_UNSUPPORTED", 7: "E_WORKSPACE"}


class afqmc_batch_options(ctypes.Structure):
    _fields_ = [("seed", c_uint64), ("n_sweep", c_int32), ("n_qr", c_int32), ("n_pc", c_int32),
                ("w_cap", c_double), ("max_branches", c_int32), ("autotune", c_int32),
                ("history", c_int32)]


class afqmc_system(ctypes.Structure):
    _fields_ = [
        ("M", c_int32), ("N", c_int32), ("n_chol", c_int32), ("K", c_int32), ("P", c_int32),
        ("hidden_kind", c_int32), ("coupling", c_double),
        ("h1", POINTER(c_double)), ("L", POINTER(c_double)), ("phi0", POINTER(c_double)),
        ("A", POINTER(c_double)),
        ("dtau", c_double), ("n_taylor", c_int32), ("weight_mode", c_int32),
        ("proposal", c_int32), ("rw_step", c_double), ("precision", c_int32),
        ("xbar_cap", c_double),
        ("trial_kind", c_int32), ("n_slices", c_int32), ("slice_s", POINTER(c_double)),
        ("slice_F", POINTER(c_double)), ("trial_taylor", c_int32),
        ("walker_c64", c_int32),
    ]


EXPORTS = {
    "afqmc_create": (c_int, [POINTER(afqmc_system), c_int, c_void_p, POINTER(c_void_p)]),
    "afqmc_destroy": (c_int, [c_void_p]),
    "afqmc_last_error": (c_char_p, [c_void_p]),
    "afqmc_set_stream": (c_int, [c_void_p, c_void_p]),
    "afqmc_workspace_size": (c_int, [c_void_p, c_int32, POINTER(c_size_t)]),
    "afqmc_set_workspace": (c_int, [c_void_p, c_void_p, c_size_t]),
    "afqmc_sample_prior": (c_int, [c_void_p, c_int32, c_uint64, c_void_p]),
    "afqmc_numeric_flags": (c_int, [c_void_p, c_int32, c_void_p, POINTER(c_int32)]),
    "afqmc_set_numeric_check": (c_int, [c_void_p, c_int32]),
    "afqmc_set_eloc_cap": (c_int, [c_void_p, c_double, c_double]),
    "afqmc_set_contraction_variant": (c_int, [c_void_p, c_int32]),
    "afqmc_trial_build": (c_int, [c_void_p, c_int32, c_void_p, c_void_p]),
    "afqmc_overlap": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "afqmc_green": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "afqmc_force_bias": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "afqmc_local_energy": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p]),
    "afqmc_local_energy_static": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p, c_void_p]),
    "afqmc_propagate": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
    "afqmc_metropolis_x": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_uint64, c_uint64, c_int32, c_void_p]),
    "afqmc_reorthogonalize": (c_int, [c_void_p, c_int32, c_void_p, c_void_p]),
    "afqmc_estimator": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "afqmc_copy": (c_int, [c_void_p, ctypes.c_int64, c_void_p, c_void_p]),
    "afqmc_gather_rows": (c_int, [c_void_p, c_int32, c_void_p, ctypes.c_int64, c_void_p, c_void_p]),
    "afqmc_bp_record": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                c_void_p]),
    "afqmc_bp_density": (c_int, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p]),
    "afqmc_init_metropolis": (c_int, [c_void_p, c_int32, c_uint64, c_int32, c_int32, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "afqmc_extend_paths": (c_int, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p]),
    "afqmc_estimator_corrected": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32,
                                          c_void_p, c_void_p, c_void_p]),
    "afqmc_population_control": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                         c_void_p, c_uint64, c_uint64, c_double, c_int32,
                                         c_void_p]),
    "afqmc_philox_normal": (c_int, [c_void_p, c_uint64, c_uint64, c_uint32, c_int32, c_int32,
                                    c_void_p]),
    "afqmc_green_diag": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "afqmc_mlp_num_params": (ctypes.c_int64, [c_void_p]),
    "afqmc_mlp_init": (c_int, [c_void_p, c_int32, POINTER(c_double), c_double, c_double, c_double,
                               c_double]),
    "afqmc_mlp_get_params": (c_int, [c_void_p, POINTER(c_double)]),
    "afqmc_mlp_set_training": (c_int, [c_void_p, c_int32]),
    "afqmc_mlp_forward": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "afqmc_mlp_train_step": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p]),
    "afqmc_batch_create": (c_int, [c_void_p, POINTER(c_int32), c_int32,
                                   POINTER(afqmc_batch_options), c_int, c_void_p,
                                   POINTER(c_void_p)]),
    "afqmc_batch_cycle": (c_int32, [c_void_p]),
    "afqmc_batch_run": (c_int, [c_void_p, c_int32]),
    "afqmc_batch_estimates": (c_int, [c_void_p, POINTER(c_double), POINTER(c_uint64)]),
    "afqmc_batch_plan": (c_int, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_double),
                                 POINTER(c_int32)]),
    "afqmc_batch_last_error": (c_char_p, [c_void_p]),
    "afqmc_batch_destroy": (c_int, [c_void_p]),
}

_lib = None


def load_library():
    """Load libafqmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2505_18519_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class AfqmcError(RuntimeError):
    def __init__(self, msg, status=None):
        super().__init__(msg)
        self.status = status


def _check(ctx, st, what):
    if st != 0:
        msg = ""
        if ctx is not None and ctx.handle:
            m = load_library().afqmc_last_error(ctx.handle)
            msg = m.decode() if m else ""
        raise AfqmcError(f"{what}: {STATUS.get(st, st)} {msg}", st)


def _ptr(t, dtype, numel, name, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return c_void_p(t.data_ptr())


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def system_struct(system, P, dtau, n_taylor=10, weight_mode=WEIGHT_SEPARATE,
                  proposal=PROPOSAL_PRIOR, rw_step=None, xbar_cap=0.0, precision=PREC_FP64,
                  walker_c64=False):
    """(afqmc_system, host arrays it points into) for a system description."""
    import numpy as np
    if rw_step is None:
        rw_step = 0.5 if proposal == PROPOSAL_RW else 0.0
    host = [np.ascontiguousarray(a, dtype=np.float64)
            for a in (system.h1, system.L, system.phi0, system.A)]
    dp = lambda a: a.ctypes.data_as(POINTER(c_double))
    st = afqmc_system(int(system.M), int(system.N), int(system.n_chol), int(system.K), int(P),
                      int(system.hidden_kind), float(system.coupling), dp(host[0]), dp(host[1]),
                      dp(host[2]), dp(host[3]), float(dtau), int(n_taylor), int(weight_mode),
                      int(proposal), float(rw_step), int(precision), float(xbar_cap))
    st.walker_c64 = 1 if walker_c64 else 0
    kind = int(getattr(system, "trial_kind", TRIAL_JASTROW))
    if kind == TRIAL_SLICES:
        s_arr = np.ascontiguousarray(system.slice_s, dtype=np.float64)
        f_arr = np.ascontiguousarray(system.slice_F, dtype=np.float64)
        host += [s_arr, f_arr]
        st.trial_kind, st.n_slices = kind, int(system.n_slices)
        st.slice_s, st.slice_F = dp(s_arr), dp(f_arr)
        st.trial_taylor = int(system.trial_taylor)
    return st, host


class Context:
    """Owns an afqmc_ctx and its workspace (a torch uint8 tensor)."""

    def __init__(self, system, P, dtau, n_taylor=10, weight_mode=WEIGHT_SEPARATE,
                 proposal=PROPOSAL_PRIOR, rw_step=None, max_walkers=1, device=0, xbar_cap=0.0,
                 precision=PREC_FP64, walker_c64=False):
        """rw_step: the random-walk step (default 0.5 for PROPOSAL_RW); with
        PROPOSAL_LEARNED a value > 0 cycles random-walk and network moves
        (default 0: network moves only).  walker_c64: walkers (every phi
        argument) are complex64 tensors."""
        lib = load_library()
        if not torch.cuda.is_available():
            raise AfqmcError("no GPU available for libafqmc")
        self.M, self.N, self.G, self.K, self.P = (int(system.M), int(system.N),
                                                  int(system.n_chol), int(system.K), int(P))
        self.sys, self._host = system_struct(system, P, dtau, n_taylor, weight_mode, proposal,
                                             rw_step, xbar_cap, precision, walker_c64)
        # element type of the walker determinants phi
        self.pdtype = torch.complex64 if walker_c64 else torch.complex128
        # element type of trial determinants: complex for multi-slice trials
        self.ctrial = int(getattr(system, "trial_kind", TRIAL_JASTROW)) == TRIAL_SLICES
        self.tdtype = torch.complex128 if self.ctrial else torch.float64
        self.dtau = float(dtau)
        self.device = torch.device("cuda", device)
        self.handle = c_void_p()
        with torch.cuda.device(self.device):
            st = lib.afqmc_create(ctypes.byref(self.sys), device, _stream(), ctypes.byref(self.handle))
        if st != 0:
            self.handle = c_void_p()
            _check(None, st, "afqmc_create")
        self.workspace = None
        self.max_walkers = 0
        self.reserve(max_walkers)

    def reserve(self, nw):
        """Make the workspace large enough for nw walkers."""
        if nw <= self.max_walkers:
            return
        n = c_size_t()
        _check(self, load_library().afqmc_workspace_size(self.handle, int(nw), ctypes.byref(n)),
               "afqmc_workspace_size")
        self.workspace = torch.empty(int(n.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        _check(self, load_library().afqmc_set_workspace(self.handle, c_void_p(aligned), int(n.value)),
               "afqmc_set_workspace")
        self.max_walkers = nw

    def close(self):
        if self.handle:
            load_library().afqmc_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, name, *args):
        lib = load_library()
        lib.afqmc_set_stream(self.handle, _stream())
        _check(self, getattr(lib, name)(self.handle, *args), name)


# --- functions with the C names -------------------------------------------------

def afqmc_numeric_flags(ctx, nw):
    """(flags [nw] int32 numpy array, number flagged); reads and clears the
    flag words (AFQMC_E_NUMERIC is reported by the count, not raised)."""
    import numpy as np
    flags = np.zeros(max(int(nw), 1), dtype=np.int32)
    n = c_int32(0)
    lib = load_library()
    lib.afqmc_set_stream(ctx.handle, _stream())
    st = lib.afqmc_numeric_flags(ctx.handle, int(nw), flags.ctypes.data_as(c_void_p),
                                 ctypes.byref(n))
    if st not in (0, E_NUMERIC):
        _check(ctx, st, "afqmc_numeric_flags")
    return flags[:int(nw)], int(n.value)


def afqmc_set_numeric_check(ctx, on):
    ctx._call("afqmc_set_numeric_check", 1 if on else 0)


def afqmc_set_contraction_variant(ctx, variant):
    """FP64 contraction of real trials on the workgroup-per-path kernels:
    0 register-resident operands, 1 operands streamed from L2."""
    ctx._call("afqmc_set_contraction_variant", int(variant))


def afqmc_set_eloc_cap(ctx, center, half_width):
    """Clip Re E_L to [center - half_width, center + half_width] in every
    later local-energy call of ctx (half_width = 0: off)."""
    ctx._call("afqmc_set_eloc_cap", float(center), float(half_width))


def afqmc_sample_prior(ctx, nw, seed, y):
    ctx._call("afqmc_sample_prior", nw, seed, _ptr(y, torch.float64, nw * ctx.P * ctx.K, "y"))


def afqmc_trial_build(ctx, nw, y, phiT):
    ctx.reserve(nw)
    ctx._call("afqmc_trial_build", nw, _ptr(y, torch.float64, nw * ctx.P * ctx.K, "y"),
              _ptr(phiT, ctx.tdtype, nw * ctx.P * ctx.M * ctx.N, "phiT"))


def afqmc_overlap(ctx, nw, phi, phiT, logov):
    c = ctx
    c._call("afqmc_overlap", nw, _ptr(phi, c.pdtype, nw * 2 * c.M * c.N, "phi"),
            _ptr(phiT, ctx.tdtype, nw * c.P * c.M * c.N, "phiT"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"))


def afqmc_green(ctx, nw, phi, phiT, logov, theta):
    c = ctx
    c._call("afqmc_green", nw, _ptr(phi, c.pdtype, nw * 2 * c.M * c.N, "phi"),
            _ptr(phiT, ctx.tdtype, nw * c.P * c.M * c.N, "phiT"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"),
            _ptr(theta, torch.complex128, nw * c.P * 2 * c.M * c.N, "theta"))


def afqmc_force_bias(ctx, nw, phiT, theta, logov, xbar, vb_sample=None):
    c = ctx
    c.reserve(nw)
    c._call("afqmc_force_bias", nw, _ptr(phiT, ctx.tdtype, nw * c.P * c.M * c.N, "phiT"),
            _ptr(theta, torch.complex128, nw * c.P * 2 * c.M * c.N, "theta"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"),
            _ptr(xbar, torch.complex128, nw * c.G, "xbar"),
            _ptr(vb_sample, torch.complex128, nw * c.P * c.G, "vb_sample", allow_none=True))


def afqmc_local_energy(ctx, nw, phiT, theta, logov, eloc, e_sample=None, xbar=None):
    c = ctx
    c.reserve(nw)
    c._call("afqmc_local_energy", nw, _ptr(phiT, ctx.tdtype, nw * c.P * c.M * c.N, "phiT"),
            _ptr(theta, torch.complex128, nw * c.P * 2 * c.M * c.N, "theta"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"),
            _ptr(eloc, torch.complex128, nw, "eloc"),
            _ptr(e_sample, torch.complex128, nw * c.P, "e_sample", allow_none=True),
            _ptr(xbar, torch.complex128, nw * c.G, "xbar", allow_none=True))


STATIC_SCRATCH_BYTES = 64 << 20   # AFQMC_STATIC_SCRATCH_BYTES


def afqmc_local_energy_static(ctx, nw, phiT, theta, logov, eloc, e_sample=None, xbar=None):
    """afqmc_local_energy with its scratch in the library's fixed per-GPU
    array: no workspace is reserved and nothing is allocated."""
    c = ctx
    c._call("afqmc_local_energy_static", nw,
            _ptr(phiT, ctx.tdtype, nw * c.P * c.M * c.N, "phiT"),
            _ptr(theta, torch.complex128, nw * c.P * 2 * c.M * c.N, "theta"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"),
            _ptr(eloc, torch.complex128, nw, "eloc"),
            _ptr(e_sample, torch.complex128, nw * c.P, "e_sample", allow_none=True),
            _ptr(xbar, torch.complex128, nw * c.G, "xbar", allow_none=True))


def afqmc_propagate(ctx, nw, phi, xi, xbar, phiT, logov, e_shift, w, ref, logov_new, eloc=None):
    c = ctx
    c.reserve(nw)
    c._call("afqmc_propagate", nw, _ptr(phi, c.pdtype, nw * 2 * c.M * c.N, "phi"),
            _ptr(xi, torch.float64, nw * c.G, "xi"),
            _ptr(xbar, torch.complex128, nw * c.G, "xbar"),
            _ptr(phiT, ctx.tdtype, nw * c.P * c.M * c.N, "phiT"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"),
            _ptr(eloc, torch.complex128, nw, "eloc", allow_none=True), float(e_shift),
            _ptr(w, torch.float64, nw, "w"), _ptr(ref, torch.complex128, nw, "ref"),
            _ptr(logov_new, torch.complex128, nw * c.P, "logov_new"))


def afqmc_metropolis_x(ctx, nw, phi, y, phiT, logov, ref, w, seed, step, n_sweep, n_accept=None):
    c = ctx
    c.reserve(nw)
    c._call("afqmc_metropolis_x", nw, _ptr(phi, c.pdtype, nw * 2 * c.M * c.N, "phi"),
            _ptr(y, torch.float64, nw * c.P * c.K, "y"),
            _ptr(phiT, ctx.tdtype, nw * c.P * c.M * c.N, "phiT"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"),
            _ptr(ref, torch.complex128, nw, "ref", allow_none=w is None),
            _ptr(w, torch.float64, nw, "w", allow_none=True),
            int(seed), int(step), int(n_sweep),
            _ptr(n_accept, torch.int32, nw, "n_accept", allow_none=True))


def afqmc_reorthogonalize(ctx, nw, phi, logov=None):
    c = ctx
    c._call("afqmc_reorthogonalize", nw, _ptr(phi, c.pdtype, nw * 2 * c.M * c.N, "phi"),
            _ptr(logov, torch.complex128, nw * c.P, "logov", allow_none=True))


def afqmc_population_control(ctx, nw, phi, w, y, phiT, logov, seed, step, w_cap=0.0, parent=None,
                             normalize=False):
    c = ctx
    c.reserve(nw)
    c._call("afqmc_population_control", nw,
            _ptr(phi, c.pdtype, nw * 2 * c.M * c.N, "phi"), _ptr(w, torch.float64, nw, "w"),
            _ptr(y, torch.float64, nw * c.P * c.K, "y"),
            _ptr(phiT, ctx.tdtype, nw * c.P * c.M * c.N, "phiT"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"), int(seed), int(step), float(w_cap),
            1 if normalize else 0, _ptr(parent, torch.int32, nw, "parent", allow_none=True))


def afqmc_estimator(ctx, nw, w, eloc, out):
    ctx._call("afqmc_estimator", nw, _ptr(w, torch.float64, nw, "w"),
              _ptr(eloc, torch.complex128, nw, "eloc"), _ptr(out, torch.float64, 2, "out"))


def _doubles(t):
    return t.numel() * (2 if t.is_complex() else 1)


def afqmc_copy(ctx, src, dst):
    """dst <- src (same size, device tensors)."""
    n = _doubles(src)
    if _doubles(dst) != n:
        raise ValueError("afqmc_copy: sizes differ")
    ctx._call("afqmc_copy", n, _ptr(src, src.dtype, src.numel(), "src"),
              _ptr(dst, dst.dtype, dst.numel(), "dst"))


def afqmc_gather_rows(ctx, nw, parent, src, dst):
    """dst[j] = src[parent[j]] over the leading (walker) dimension."""
    row = _doubles(src) // nw
    if _doubles(dst) != row * nw or _doubles(src) != row * nw:
        raise ValueError("afqmc_gather_rows: sizes differ")
    ctx._call("afqmc_gather_rows", nw, _ptr(parent, torch.int32, nw, "parent"), row,
              _ptr(src, src.dtype, src.numel(), "src"), _ptr(dst, dst.dtype, dst.numel(), "dst"))


def afqmc_bp_record(ctx, nw, h, slot, xi, xbar, hist_xi, hist_xbar):
    c = ctx
    c._call("afqmc_bp_record", nw, int(h), int(slot), _ptr(xi, torch.float64, nw * c.G, "xi"),
            _ptr(xbar, torch.complex128, nw * c.G, "xbar"),
            _ptr(hist_xi, torch.float64, nw * h * c.G, "hist_xi"),
            _ptr(hist_xbar, torch.complex128, nw * h * c.G, "hist_xbar"))


def afqmc_bp_density(ctx, nw, h, phi_mid, hist_xi, hist_xbar, phiT, logov, w, phit_bp, theta_bp,
                     logov_bp, rho, out):
    c = ctx
    c.reserve(nw)
    c._call("afqmc_bp_density", nw, int(h),
            _ptr(phi_mid, torch.complex128, nw * 2 * c.M * c.N, "phi_mid"),
            _ptr(hist_xi, torch.float64, nw * h * c.G, "hist_xi", allow_none=h == 0),
            _ptr(hist_xbar, torch.complex128, nw * h * c.G, "hist_xbar", allow_none=h == 0),
            _ptr(phiT, ctx.tdtype, nw * c.P * c.M * c.N, "phiT"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"), _ptr(w, torch.float64, nw, "w"),
            _ptr(phit_bp, torch.complex128, nw * c.P * c.M * c.N, "phit_bp"),
            _ptr(theta_bp, torch.complex128, nw * c.P * 2 * c.M * c.N, "theta_bp"),
            _ptr(logov_bp, torch.complex128, nw * c.P, "logov_bp"),
            _ptr(rho, torch.complex128, nw * c.M * c.M, "rho"),
            _ptr(out, torch.float64, c.M * c.M + 1, "out"))


def afqmc_init_metropolis(ctx, nw, seed, n_pair, n_burn, yw, phi, y, phiT, logov, w):
    c = ctx
    c.reserve(nw)
    c._call("afqmc_init_metropolis", nw, int(seed), int(n_pair), int(n_burn),
            _ptr(yw, torch.float64, nw * c.K, "yw"),
            _ptr(phi, c.pdtype, nw * 2 * c.M * c.N, "phi"),
            _ptr(y, torch.float64, nw * c.P * c.K, "y"),
            _ptr(phiT, ctx.tdtype, nw * c.P * c.M * c.N, "phiT"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"), _ptr(w, torch.float64, nw, "w"))


def afqmc_extend_paths(ctx, nw, p_src, y_src, phiT_src, logov_src, y, phiT, logov):
    c = ctx
    c._call("afqmc_extend_paths", nw, int(p_src),
            _ptr(y_src, torch.float64, nw * p_src * c.K, "y_src"),
            _ptr(phiT_src, ctx.tdtype, nw * p_src * c.M * c.N, "phiT_src"),
            _ptr(logov_src, torch.complex128, nw * p_src, "logov_src"),
            _ptr(y, torch.float64, nw * c.P * c.K, "y"),
            _ptr(phiT, ctx.tdtype, nw * c.P * c.M * c.N, "phiT"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"))


def afqmc_estimator_corrected(ctx, nw, w, eloc, logov, p_ref, logov_ref, out, R=None):
    c = ctx
    c._call("afqmc_estimator_corrected", nw, _ptr(w, torch.float64, nw, "w"),
            _ptr(eloc, torch.complex128, nw, "eloc"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"), int(p_ref),
            _ptr(logov_ref, torch.complex128, nw * p_ref, "logov_ref"),
            _ptr(out, torch.float64, 2, "out"),
            _ptr(R, torch.complex128, nw, "R", allow_none=True))


def afqmc_philox_normal(ctx, seed, step, tag, nw, n, out):
    ctx._call("afqmc_philox_normal", int(seed), int(step), int(tag), nw, n,
              _ptr(out, torch.float64, nw * n, "out"))


def afqmc_green_diag(ctx, nw, phi, phiT, logov, gdiag):
    c = ctx
    c._call("afqmc_green_diag", nw, _ptr(phi, c.pdtype, nw * 2 * c.M * c.N, "phi"),
            _ptr(phiT, ctx.tdtype, nw * c.P * c.M * c.N, "phiT"),
            _ptr(logov, torch.complex128, nw * c.P, "logov"),
            _ptr(gdiag, torch.float64, nw * c.P * c.M, "gdiag"))


# --- learned proposal network ---------------------------------------------------

def afqmc_mlp_num_params(ctx):
    return int(load_library().afqmc_mlp_num_params(ctx.handle))


MLP_PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def mlp_pack(params):
    """The flat parameter array of afqmc_mlp_init from a dict of the six
    network arrays: W1 [D][H], b1 [H], W2 [H][H], b2 [H], W3 [H][2K], b3 [2K],
    each row-major, concatenated in that order (the layout afqmc.h states)."""
    import numpy as np
    return np.concatenate([np.asarray(params[k], dtype=np.float64).ravel()
                           for k in MLP_PARAM_ORDER])


def afqmc_mlp_init(ctx, precision, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """params: host float64 array of afqmc_mlp_num_params(ctx) values, or a
    dict of the six arrays (packed by mlp_pack)."""
    import numpy as np
    if isinstance(params, dict):
        params = mlp_pack(params)
    p = np.ascontiguousarray(params, dtype=np.float64).ravel()
    n = afqmc_mlp_num_params(ctx)
    if p.size != n:
        raise ValueError(f"params has {p.size} values, the network has {n}")
    ctx._call("afqmc_mlp_init", int(precision), p.ctypes.data_as(POINTER(c_double)), float(lr),
              float(beta1), float(beta2), float(eps))


def afqmc_mlp_get_params(ctx):
    import numpy as np
    out = np.empty(afqmc_mlp_num_params(ctx), dtype=np.float64)
    ctx._call("afqmc_mlp_get_params", out.ctypes.data_as(POINTER(c_double)))
    return out


def afqmc_mlp_set_training(ctx, enabled):
    ctx._call("afqmc_mlp_set_training", 1 if enabled else 0)


def afqmc_mlp_forward(ctx, n, gdiag, y, mu, lv):
    c = ctx
    c.reserve((n + c.P - 1) // c.P)
    c._call("afqmc_mlp_forward", n, _ptr(gdiag, torch.float64, n * c.M, "gdiag"),
            _ptr(y, torch.float64, n * c.K, "y"), _ptr(mu, torch.float64, n * c.K, "mu"),
            _ptr(lv, torch.float64, n * c.K, "lv"))


def afqmc_mlp_train_step(ctx, n, gdiag, y, ytarget, mask, loss=None, grad=None):
    c = ctx
    c.reserve((n + c.P - 1) // c.P)
    c._call("afqmc_mlp_train_step", n, _ptr(gdiag, torch.float64, n * c.M, "gdiag"),
            _ptr(y, torch.float64, n * c.K, "y"), _ptr(ytarget, torch.float64, n * c.K, "ytarget"),
            _ptr(mask, torch.int32, n, "mask"),
            _ptr(loss, torch.float64, 1, "loss", allow_none=True),
            _ptr(grad, torch.float64, afqmc_mlp_num_params(c), "grad", allow_none=True))


# --- uneven batching ---------------------------------------------------------------

class Batch:
    """Owns an afqmc_batch: systems [(system, P, dtau, kwargs)], walkers per system."""

    def __init__(self, systems, walkers, seed, n_sweep=1, n_qr=10, n_pc=1, w_cap=0.0,
                 max_branches=4, autotune=True, history=256, device=0):
        import numpy as np
        lib = load_library()
        if not torch.cuda.is_available():
            raise AfqmcError("no GPU available for libafqmc")
        self.n = len(systems)
        structs, self._host = [], []
        for (system, P, dtau, kw) in systems:
            st, host = system_struct(system, P, dtau, **kw)
            structs.append(st)
            self._host.append(host)
        self._arr = (afqmc_system * self.n)(*structs)
        self._walkers = (c_int32 * self.n)(*[int(w) for w in walkers])
        self.history = int(history)
        self.opt = afqmc_batch_options(int(seed), int(n_sweep), int(n_qr), int(n_pc), float(w_cap),
                                       int(max_branches), 1 if autotune else 0, self.history)
        self.handle = c_void_p()
        with torch.cuda.device(device):
            rc = lib.afqmc_batch_create(ctypes.cast(self._arr, c_void_p), self._walkers, self.n,
                                        ctypes.byref(self.opt), device, _stream(),
                                        ctypes.byref(self.handle))
        if rc != 0:
            self.handle = c_void_p()
            raise AfqmcError(f"afqmc_batch_create: {STATUS.get(rc, rc)}")
        self.cycle = int(lib.afqmc_batch_cycle(self.handle))

    def _check(self, rc, what):
        if rc != 0:
            m = load_library().afqmc_batch_last_error(self.handle)
            raise AfqmcError(f"{what}: {STATUS.get(rc, rc)} {m.decode() if m else ''}")

    def run(self, n_cycles):
        self._check(load_library().afqmc_batch_run(self.handle, int(n_cycles)), "afqmc_batch_run")

    def estimates(self):
        """(sums [n][history][2], steps [n]) for the ring of the last `history` steps."""
        import numpy as np
        out = np.zeros((self.n, self.history, 2))
        steps = np.zeros(self.n, dtype=np.uint64)
        self._check(load_library().afqmc_batch_estimates(
            self.handle, out.ctypes.data_as(POINTER(c_double)),
            steps.ctypes.data_as(POINTER(c_uint64))), "afqmc_batch_estimates")
        return out, steps

    def plan(self):
        import numpy as np
        fam = np.zeros(self.n, dtype=np.int32)
        br = np.zeros(self.n, dtype=np.int32)
        ms = np.zeros(self.n)
        nb = c_int32()
        self._check(load_library().afqmc_batch_plan(
            self.handle, fam.ctypes.data_as(POINTER(c_int32)), br.ctypes.data_as(POINTER(c_int32)),
            ms.ctypes.data_as(POINTER(c_double)), ctypes.byref(nb)), "afqmc_batch_plan")
        return fam, br, ms, int(nb.value)

    def close(self):
        if self.handle:
            load_library().afqmc_batch_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
