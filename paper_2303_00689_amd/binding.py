"""ctypes binding of libxlbomd (argument marshalling only).

Each method forwards torch device tensors (their data pointers) to the C ABI
declared in include/xlbomd.h.  No arithmetic of the method happens here.  The
library must have been built (``python -m paper_2303_00689_amd.build`` or
``__graft_entry__.build()``); loading fails loudly otherwise.
"""

from __future__ import annotations

import ctypes as C
import math
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxlbomd.so")

PREC = {"fp64": 0, "bf16x3": 1, "bf16x6": 2, "fp16x3": 3,
        "dm64_bf16x3": 4, "dm64_bf16x6": 5, "dm64_fp16x3": 6}

STATUS = {0: "OK", -1: "E_ARG", -2: "E_HIP", -3: "E_NOCONV", -4: "E_NONFINITE",
          -5: "E_STATE", -6: "E_NOMEM", -7: "E_UNSTABLE"}

# symbols declared in include/xlbomd.h
SYMBOLS = ["xlbomd_create", "xlbomd_destroy", "xlbomd_last_error", "xlbomd_n_orb",
           "xlbomd_set_geometry", "xlbomd_hcore", "xlbomd_fock", "xlbomd_fermi_dm", "xlbomd_spectral_bounds",
           "xlbomd_dm_response", "xlbomd_krylov_kernel", "xlbomd_forces", "xlbomd_integrate",
           "xlbomd_step", "xlbomd_step_langevin", "xlbomd_ensemble_step", "xlbomd_md_init", "xlbomd_scf",
           "xlbomd_matmul",
           "xlbomd_profile", "xlbomd_profile_read", "xlbomd_spectral_bounds_noalloc",
           "xlbomd_set_tile_table", "xlbomd_time_gemm",
           "xlbomd_overlap", "xlbomd_lowdin", "xlbomd_fermi_dm_nonorth", "xlbomd_dm_response_nonorth",
           "xlbomd_pulay_forces"]

# GEMM kernel families of the tile table (xlbomd_set_tile_table)
GEMM_AUTO, GEMM_SMALL, GEMM_LARGE, GEMM_MEDIUM, GEMM_COMPACT = 0, 1, 2, 3, 4
TILE_TABLE_MAX = 256
# the tile table the autotuner wrote (autotune.py), loaded with the library;
# XLBOMD_TILE_TABLE names another file, or "none" for the built-in rule
TILE_TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_table.json")

# largest n of xlbomd_spectral_bounds_noalloc (XLBOMD_SPECTRAL_BOUNDS_NOALLOC_MAX_N)
SPECTRAL_BOUNDS_NOALLOC_MAX_N = 16384


class OverlapModelC(C.Structure):
    _fields_ = [("s0", C.c_double), ("r0", C.c_double), ("lam", C.c_double)]


class Model(C.Structure):
    _fields_ = [(name, C.c_double) for name in
                ("eps_s", "eps_p", "t0", "r0_hop", "lam_hop", "coul_k", "coul_a", "noise_amp",
                 "z_core", "a_rep", "r0_rep", "rho_rep", "mass")] + [("j55", C.c_double * 55)]


class System(C.Structure):
    _fields_ = [("n_atoms", C.c_int), ("n_elec", C.c_double),
                ("onecenter", C.POINTER(C.c_double)), ("noise55", C.POINTER(C.c_float)),
                ("model", Model)]


class Params(C.Structure):
    _fields_ = [("prec", C.c_int), ("T_e", C.c_double), ("m", C.c_int), ("krylov_tol", C.c_double),
                ("dt", C.c_double), ("kappa", C.c_double), ("alpha", C.c_double),
                ("c", C.c_double * 7), ("kernel_c", C.c_double), ("w0_limit", C.c_double),
                ("T_ion_limit", C.c_double)]


class MDStateC(C.Structure):
    _fields_ = [("R", C.c_void_p), ("V", C.c_void_p), ("A", C.c_void_p), ("X", C.c_void_p),
                ("Y", C.c_void_p), ("head", C.c_int), ("mu", C.c_double), ("mu_prev", C.c_double)]


class SCFParams(C.Structure):
    _fields_ = [("m", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int), ("mix", C.c_double),
                ("mix_tol", C.c_double), ("max_mix", C.c_int)]


class SCFReport(C.Structure):
    _fields_ = [("residual", C.c_double), ("mix_steps", C.c_int), ("newton_steps", C.c_int),
                ("evaluations", C.c_int), ("responses", C.c_int)]


class Report(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("E_tot", "KE", "U", "TS", "T_ion", "mu", "W0", "relres")] + \
               [("rank", C.c_int), ("status", C.c_int), ("levels", C.c_int), ("mu_passes", C.c_int)]


_lib = None


def load():
    """Load libxlbomd.so and declare the prototypes."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    pd = C.POINTER(C.c_double)
    pi = C.POINTER(C.c_int)
    lib.xlbomd_create.argtypes = [C.POINTER(System), C.POINTER(Params), vp, C.POINTER(vp)]
    lib.xlbomd_destroy.argtypes = [vp]
    lib.xlbomd_last_error.argtypes = [vp]
    lib.xlbomd_last_error.restype = C.c_char_p
    lib.xlbomd_n_orb.argtypes = [vp]
    lib.xlbomd_n_orb.restype = i
    lib.xlbomd_set_geometry.argtypes = [vp, vp]
    lib.xlbomd_hcore.argtypes = [vp, vp]
    lib.xlbomd_fock.argtypes = [vp, vp, vp, i]
    lib.xlbomd_fermi_dm.argtypes = [vp, vp, pd, vp, pd]
    lib.xlbomd_spectral_bounds.argtypes = [vp, vp, pd]
    lib.xlbomd_dm_response.argtypes = [vp, vp, vp]
    lib.xlbomd_krylov_kernel.argtypes = [vp, vp, vp, i, d, vp, pi, pd]
    lib.xlbomd_forces.argtypes = [vp, vp, vp, vp, pd]
    lib.xlbomd_integrate.argtypes = [vp, C.POINTER(MDStateC)]
    lib.xlbomd_step.argtypes = [vp, C.POINTER(MDStateC), i, C.POINTER(Report)]
    lib.xlbomd_step_langevin.argtypes = [vp, C.POINTER(MDStateC), i, d, d, vp, C.POINTER(Report)]
    lib.xlbomd_ensemble_step.argtypes = [C.POINTER(vp), C.POINTER(MDStateC), i, i, C.POINTER(Report)]
    lib.xlbomd_md_init.argtypes = [vp, C.POINTER(MDStateC)]
    lib.xlbomd_scf.argtypes = [vp, vp, C.POINTER(SCFParams), pd, i, C.POINTER(SCFReport)]
    lib.xlbomd_matmul.argtypes = [vp, vp, vp, vp, i, i]
    lib.xlbomd_profile.argtypes = [vp, i]
    lib.xlbomd_profile_read.argtypes = [vp, pd]
    lib.xlbomd_spectral_bounds_noalloc.argtypes = [vp, i, vp, pd]
    lib.xlbomd_set_tile_table.argtypes = [pi, i]
    lib.xlbomd_time_gemm.argtypes = [i, i, i, i, i, vp, pd]
    ovp = C.POINTER(OverlapModelC)
    lib.xlbomd_overlap.argtypes = [vp, ovp, vp]
    lib.xlbomd_lowdin.argtypes = [vp, vp, vp, pi]
    lib.xlbomd_fermi_dm_nonorth.argtypes = [vp, vp, vp, pd, vp, pd]
    lib.xlbomd_dm_response_nonorth.argtypes = [vp, vp, vp, vp]
    lib.xlbomd_pulay_forces.argtypes = [vp, ovp, vp, vp, vp, vp]
    for name in SYMBOLS:
        if name not in ("xlbomd_last_error", "xlbomd_n_orb"):
            getattr(lib, name).restype = i
    _lib = lib
    install_tile_table()
    return lib


def install_tile_table():
    """Install the default tile table: the file XLBOMD_TILE_TABLE names, else
    the autotuner's tile_table.json beside this module; none (the built-in
    rule) if XLBOMD_TILE_TABLE is "none" or the file is absent."""
    path = os.environ.get("XLBOMD_TILE_TABLE", TILE_TABLE_PATH)
    rows = []
    if path != "none" and os.path.exists(path):
        with open(path) as f:
            rows = json.load(f)["rows"]
    set_tile_table(rows)


def set_tile_table(rows):
    """Install the GEMM tile table: rows of (prec, sym, n_max, family), prec
    0..3 = FP64, BF16x3, BF16x6, FP16x3 (xlbomd_set_tile_table); [] clears it."""
    lib = load()
    flat = [int(v) for r in rows for v in r]
    if len(flat) != 4 * len(rows):
        raise XLBOMDError("tile table rows must have 4 entries")
    arr = (C.c_int * max(len(flat), 1))(*flat)
    st = lib.xlbomd_set_tile_table(arr, len(rows))
    if st != 0:
        raise XLBOMDError(f"set_tile_table: {STATUS.get(st, st)}", st)


def time_gemm(n, prec, sym, family, reps=5, stream=None):
    """Microseconds per n x n product of kernel family `family` (xlbomd_time_gemm),
    or None if the family cannot run n."""
    lib = load()
    us = C.c_double(0.0)
    st = lib.xlbomd_time_gemm(int(n), int(prec), int(sym), int(family), int(reps), C.c_void_p(stream or 0),
                              C.byref(us))
    if st == -1:
        return None
    if st != 0:
        raise XLBOMDError(f"time_gemm: {STATUS.get(st, st)}", st)
    return us.value


class XLBOMDError(RuntimeError):
    """A library call failed; .status holds its xlbomd_status (None for
    argument checks of the binding itself)."""

    def __init__(self, msg, status=None):
        super().__init__(msg)
        self.status = status


def _ptr(t, n_elem=None, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise XLBOMDError("expected a device tensor")
    if not t.is_contiguous():
        raise XLBOMDError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise XLBOMDError(f"expected dtype {dtype}, got {t.dtype}")
    if n_elem is not None and t.numel() != n_elem:
        raise XLBOMDError(f"expected {n_elem} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class MDState:
    """Device state of xlbomd_step (R, V, A: N x 3; X: 7 x n x n ring; Y: n x n)
    and its host fields (ring head, the last two chemical potentials)."""

    def __init__(self, R, V, A, X, Y, head=0, mu=float("nan"), mu_prev=float("nan")):
        self.R, self.V, self.A, self.X, self.Y = R, V, A, X, Y
        self.head, self.mu, self.mu_prev = head, mu, mu_prev

    def _c(self, h):
        import torch
        N, n = h.n_atoms, h.n
        f = torch.float64
        return MDStateC(_ptr(self.R, 3 * N, f), _ptr(self.V, 3 * N, f), _ptr(self.A, 3 * N, f),
                        _ptr(self.X, 7 * n * n, f), _ptr(self.Y, n * n, f), self.head, self.mu, self.mu_prev)

    def _back(self, sc):
        self.head, self.mu, self.mu_prev = sc.head, sc.mu, sc.mu_prev

    def x_current(self):
        return self.X[self.head]


class Handle:
    """One system on the current device (see include/xlbomd.h for semantics)."""

    def __init__(self, n_atoms, n_elec, onecenter, noise55, model, *, prec="fp64", T_e=3000.0,
                 m=4, dt=0.5, kappa=1.84, alpha=0.0055,
                 c=(-14.0, 36.0, -27.0, -2.0, 12.0, -6.0, 1.0), krylov_tol=0.0, kernel_c=1.0, w0_limit=0.0,
                 T_ion_limit=0.0, stream=None):
        self.lib = load()
        self.n_atoms = int(n_atoms)
        self.n = 4 * self.n_atoms
        self._oc = np.ascontiguousarray(onecenter, dtype=np.float64)
        if self._oc.shape != (self.n_atoms, 5):
            raise XLBOMDError("onecenter must be (n_atoms, 5)")
        npair = self.n_atoms * (self.n_atoms - 1) // 2
        # the ABI takes the noise blocks in FP32: values that FP32 does not hold
        # exactly are refused rather than rounded
        noise = np.asarray(noise55) if npair else np.zeros((0, 55), np.float32)
        self._noise = np.ascontiguousarray(noise, dtype=np.float32)
        if noise.dtype != np.float32 and not np.array_equal(self._noise.astype(noise.dtype), noise):
            raise XLBOMDError("noise55 holds values that FP32 does not represent exactly")
        if self._noise.shape != (npair, 55):
            raise XLBOMDError("noise55 must be (n_pair, 55)")
        mdl = Model()
        for name, _ in Model._fields_[:-1]:
            setattr(mdl, name, float(getattr(model, name)))
        j = np.asarray(model.j55(), dtype=np.float64)
        for k in range(55):
            mdl.j55[k] = j[k]
        sysc = System(self.n_atoms, float(n_elec), self._oc.ctypes.data_as(C.POINTER(C.c_double)),
                      self._noise.ctypes.data_as(C.POINTER(C.c_float)), mdl)
        prm = Params(PREC[prec] if isinstance(prec, str) else int(prec), float(T_e), int(m),
                     float(krylov_tol), float(dt), float(kappa), float(alpha), (C.c_double * 7)(*c),
                     float(kernel_c), float(w0_limit), float(T_ion_limit))
        self.prec = prec
        self.m = int(m)
        h = C.c_void_p()
        st = self.lib.xlbomd_create(C.byref(sysc), C.byref(prm), C.c_void_p(stream or 0), C.byref(h))
        if st != 0:
            raise XLBOMDError(f"xlbomd_create failed: {STATUS.get(st, st)}")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.xlbomd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            msg = self.lib.xlbomd_last_error(self.h).decode()
            raise XLBOMDError(f"{what}: {STATUS.get(st, st)}: {msg}", st)

    def _mat(self, t):
        import torch
        return _ptr(t, self.n * self.n, torch.float64)

    def set_geometry(self, R):
        import torch
        self._check(self.lib.xlbomd_set_geometry(self.h, _ptr(R, 3 * self.n_atoms, torch.float64)),
                    "set_geometry")

    def hcore(self, H):
        self._check(self.lib.xlbomd_hcore(self.h, self._mat(H)), "hcore")

    def fock(self, P, F, include_h=True):
        self._check(self.lib.xlbomd_fock(self.h, self._mat(P), self._mat(F), int(bool(include_h))), "fock")

    def fermi_dm(self, F, P, mu=float("nan"), entropy=True):
        """(mu, S/k_B); entropy=False skips the entropy's eigenvalue solve (S = nan)."""
        m = C.c_double(mu)
        S = C.c_double(float("nan"))
        self._check(self.lib.xlbomd_fermi_dm(self.h, self._mat(F), C.byref(m), self._mat(P),
                                             C.byref(S) if entropy else None), "fermi_dm")
        return m.value, S.value

    def spectral_bounds(self, F):
        """(lo, hi) enclosing the spectrum of F (the chain-depth step)."""
        lohi = (C.c_double * 2)()
        self._check(self.lib.xlbomd_spectral_bounds(self.h, self._mat(F), lohi), "spectral_bounds")
        return lohi[0], lohi[1]

    def dm_response(self, F1, P1):
        self._check(self.lib.xlbomd_dm_response(self.h, self._mat(F1), self._mat(P1)), "dm_response")

    def krylov_kernel(self, X, P0, m, Y, tol=0.0):
        r = C.c_int(0)
        rel = C.c_double(0.0)
        self._check(self.lib.xlbomd_krylov_kernel(self.h, self._mat(X), self._mat(P0), int(m), float(tol),
                                                  self._mat(Y), C.byref(r), C.byref(rel)), "krylov_kernel")
        return r.value, rel.value

    def forces(self, P0, X, frc):
        import torch
        e = (C.c_double * 4)()
        self._check(self.lib.xlbomd_forces(self.h, self._mat(P0), self._mat(X),
                                           _ptr(frc, 3 * self.n_atoms, torch.float64), e), "forces")
        return list(e)

    # ---- non-orthogonal basis (ov: any object with s0, r0, lam)
    @staticmethod
    def _ov(ov):
        return C.byref(OverlapModelC(float(ov.s0), float(ov.r0), float(ov.lam)))

    def overlap(self, ov, S):
        self._check(self.lib.xlbomd_overlap(self.h, self._ov(ov), self._mat(S)), "overlap")

    def lowdin(self, S, Z):
        """Z = S^(-1/2); returns the Newton-Schulz iteration count."""
        it = C.c_int(0)
        self._check(self.lib.xlbomd_lowdin(self.h, self._mat(S), self._mat(Z), C.byref(it)), "lowdin")
        return it.value

    def fermi_dm_nonorth(self, F, Z, P, mu=float("nan"), entropy=True):
        """(mu, S/k_B) as fermi_dm."""
        m = C.c_double(mu)
        S = C.c_double(float("nan"))
        self._check(self.lib.xlbomd_fermi_dm_nonorth(self.h, self._mat(F), self._mat(Z), C.byref(m), self._mat(P),
                                                     C.byref(S) if entropy else None), "fermi_dm_nonorth")
        return m.value, S.value

    def dm_response_nonorth(self, F1, Z, P1):
        self._check(self.lib.xlbomd_dm_response_nonorth(self.h, self._mat(F1), self._mat(Z), self._mat(P1)),
                    "dm_response_nonorth")

    def pulay_forces(self, ov, F, P, Z, frc):
        import torch
        self._check(self.lib.xlbomd_pulay_forces(self.h, self._ov(ov), self._mat(F), self._mat(P), self._mat(Z),
                                                 _ptr(frc, 3 * self.n_atoms, torch.float64)), "pulay_forces")

    def integrate(self, state: MDState):
        sc = state._c(self)
        self._check(self.lib.xlbomd_integrate(self.h, C.byref(sc)), "integrate")
        state._back(sc)

    def md_init(self, state: MDState):
        sc = state._c(self)
        self._check(self.lib.xlbomd_md_init(self.h, C.byref(sc)), "md_init")
        state._back(sc)

    def step(self, state: MDState, n_steps=1, report=True, check=True):
        """n_steps NVE steps; returns the per-step reports (report=True).  With
        check=False a failing call returns (status, reports) instead of raising:
        the failing step's report carries the status."""
        sc = state._c(self)
        reps = (Report * max(n_steps, 1))() if report or not check else None
        st = self.lib.xlbomd_step(self.h, C.byref(sc), int(n_steps), reps)
        state._back(sc)
        out = None if reps is None else [{k: getattr(r, k) for k, _ in Report._fields_} for r in reps[:n_steps]]
        if not check:
            return st, out
        self._check(st, "step")
        return out if report else None

    def step_langevin(self, state: MDState, xi, gamma, T_ion, report=True):
        """len(xi) / (3 n_atoms) Langevin steps; xi: device float64 standard normals."""
        import torch
        if (not isinstance(xi, torch.Tensor) or not xi.is_cuda or xi.dtype != torch.float64
                or not xi.is_contiguous() or xi.numel() % (3 * self.n_atoms)):
            raise XLBOMDError("xi must be a contiguous float64 device tensor of n_steps x n_atoms x 3")
        n_steps = xi.numel() // (3 * self.n_atoms)
        sc = state._c(self)
        reps = (Report * max(n_steps, 1))() if report else None
        self._check(self.lib.xlbomd_step_langevin(self.h, C.byref(sc), int(n_steps), float(gamma), float(T_ion),
                                                  C.c_void_p(xi.data_ptr()), reps), "step_langevin")
        state._back(sc)
        if not report:
            return None
        return [{k: getattr(r, k) for k, _ in Report._fields_} for r in reps[:n_steps]]

    def matmul(self, A, B, Cout, sym_out=False, reps=1):
        self._check(self.lib.xlbomd_matmul(self.h, self._mat(A), self._mat(B), self._mat(Cout),
                                           int(bool(sym_out)), int(reps)), "matmul")

    def profile(self, enable=True):
        self._check(self.lib.xlbomd_profile(self.h, int(bool(enable))), "profile")

    PROFILE_CLASSES = ("gemm_f64", "gemm_f64_sym", "gemm_bf16x3", "gemm_bf16x3_sym", "gemm_bf16x6",
                       "gemm_bf16x6_sym", "gemm_fp16x3", "gemm_fp16x3_sym", "fock", "forces")

    def profile_read(self):
        """Per kernel class: launches, milliseconds and work (see xlbomd_profile_read)."""
        out = (C.c_double * 30)()
        self._check(self.lib.xlbomd_profile_read(self.h, out), "profile_read")
        return {nm: dict(launches=int(out[3 * k]), ms=out[3 * k + 1], work=out[3 * k + 2])
                for k, nm in enumerate(self.PROFILE_CLASSES)}

    def scf(self, X, m=20, tol=1e-10, max_iter=100, mix=0.04, mix_tol=1e-2, max_mix=5000,
            allow_noconv=False, history=0):
        """Ground state into X (xlbomd_scf).  Returns a dict with the final
        residual ||D0[X] - X||_F, the mixing and Newton steps taken, the
        density-matrix evaluations and responses, and (history > 0) the first
        `history` residuals.  With allow_noconv a run that stops above tol
        returns its report instead of raising."""
        prm = SCFParams(int(m), float(tol), int(max_iter), float(mix), float(mix_tol), int(max_mix))
        rep = SCFReport()
        hist = (C.c_double * max(int(history), 1))()
        st = self.lib.xlbomd_scf(self.h, self._mat(X), C.byref(prm), hist if history else None,
                                 int(history), C.byref(rep))
        if not (allow_noconv and st == -3):
            self._check(st, "scf")
        out = {k: getattr(rep, k) for k, _ in SCFReport._fields_}
        if history:
            nh = min(int(history), rep.mix_steps + rep.newton_steps + 1)
            out["history"] = list(hist[:nh])
        return out


def ensemble_step(handles, states, n_steps=1, report=True):
    """Advance every (handle, state) pair by n_steps concurrently
    (xlbomd_ensemble_step); returns one list of reports per member."""
    count = len(handles)
    if len(states) != count:
        raise XLBOMDError("one state per handle")
    if count == 0:
        return []
    lib = handles[0].lib
    hs = (C.c_void_p * count)(*[h.h for h in handles])
    scs = (MDStateC * count)(*[s._c(h) for h, s in zip(handles, states)])
    reps = (Report * max(count * n_steps, 1))() if report else None
    st = lib.xlbomd_ensemble_step(hs, scs, int(count), int(n_steps), reps)
    for k, (h, s) in enumerate(zip(handles, states)):
        s._back(scs[k])
    if st != 0:
        msgs = "; ".join(f"member {k}: {h.lib.xlbomd_last_error(h.h).decode()}" for k, h in enumerate(handles)
                         if h.lib.xlbomd_last_error(h.h))
        raise XLBOMDError(f"ensemble_step failed: {STATUS.get(st, st)} ({msgs})")
    if not report:
        return None
    return [[{k: getattr(reps[m * n_steps + j], k) for k, _ in Report._fields_} for j in range(n_steps)]
            for m in range(count)]


def spectral_bounds_noalloc(F, stream=None):
    """(lo, hi) enclosing the spectrum of the symmetric n x n FP64 device
    tensor F, from xlbomd_spectral_bounds_noalloc (no handle, no allocation)."""
    import torch
    lib = load()
    if not isinstance(F, torch.Tensor) or F.dim() != 2 or F.shape[0] != F.shape[1]:
        raise XLBOMDError("F must be a square device tensor")
    n = F.shape[0]
    lohi = (C.c_double * 2)()
    st = lib.xlbomd_spectral_bounds_noalloc(_ptr(F, n * n, torch.float64), int(n), C.c_void_p(stream or 0), lohi)
    if st != 0:
        raise XLBOMDError(f"spectral_bounds_noalloc: {STATUS.get(st, st)}")
    return lohi[0], lohi[1]


def handle_for(system, settings: dict, prec="fp64", stream=None) -> Handle:
    """Handle for a synthetic cluster (``synth.System``) with workload settings."""
    return Handle(system.n_atoms, system.n_elec, system.onecenter, system.noise, system.params,
                  prec=prec, T_e=settings["T_e"], m=settings["m"], dt=settings["dt"], stream=stream)
