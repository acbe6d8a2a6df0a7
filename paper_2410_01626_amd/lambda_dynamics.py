"""Python binding of the lambda-dynamics calls of libfmmcph (argument
marshalling only: every step runs in the library's HIP kernels), and a small
driver that advances the lambda particles of a plan's sites around each
Coulomb solve (constant-pH paper, Methods: eq 1 and eq 3, "Constant pH
Parameters", "Partition Function Correction", "Dynamic Barrier and Well
Optimization")."""
from __future__ import annotations

import ctypes
import math

from .fmm import FMM_OK, FmmError, load_library

__all__ = ["LambdaParams", "DboParams", "lambda_step", "lambda_dbo", "lambda_pfc",
           "LambdaDynamics", "KB"]

KB = 8.314462618e-3  # kJ mol^-1 K^-1


class LambdaParams(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("dt", ctypes.c_double),
                ("temperature", ctypes.c_double), ("tau", ctypes.c_double),
                ("near0", ctypes.c_double), ("near1", ctypes.c_double)]


class DboParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "near0", "near1", "occupancy", "well_tol", "well_gain", "max_shift", "target",
        "target_tol", "barrier_step", "barrier_min", "barrier_max")]


def _p(t):
    return ctypes.c_void_p(0) if t is None else ctypes.c_void_p(t.data_ptr())


def _check(t, n, dtype, name, optional=False):
    import torch
    if t is None:
        if optional:
            return
        raise ValueError("%s is required" % name)
    if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise ValueError("%s: expected a contiguous %s CUDA tensor of %d elements, got %s %s %s"
                         % (name, dtype, n, t.dtype, tuple(t.shape), t.device))
    del torch


def _raise(st, name):
    if st != FMM_OK:
        raise FmmError(st, name)


def lambda_step(coord_off, lam, lam_new, v, dvdl, ph, params: LambdaParams, first=False,
                partner=None, pka=None, mm=None, dwp=None, noise=None, stats_w=None,
                stats_b=None, kin=None, e_bias=None, stream=None, check=True, dwp2=None,
                stats_b2=None):
    """fmm_lambda_step on device tensors (float64; coord_off, partner int32).
    check=False skips the checks of every tensor but dvdl (for a caller that
    has already made them on the same tensors)."""
    import torch
    R = coord_off.numel() - 1
    C = lam.numel()
    if not check:
        _check(dvdl, C, torch.float64, "dvdl")
        s = stream if stream is not None else torch.cuda.current_stream(lam.device)
        st = load_library().fmm_lambda_step(
            ctypes.c_void_p(s.cuda_stream), R, _p(coord_off), C, ctypes.byref(params),
            1 if first else 0, _p(lam), _p(lam_new), _p(v), _p(dvdl), _p(partner), _p(pka), _p(ph),
            _p(mm), _p(dwp), _p(noise), _p(stats_w), _p(stats_b), _p(kin), _p(e_bias), _p(dwp2),
            _p(stats_b2))
        _raise(st, "fmm_lambda_step")
        return
    f64, i32 = torch.float64, torch.int32
    _check(coord_off, R + 1, i32, "coord_off")
    for t, n, nm in ((lam, C, "lam"), (lam_new, C, "lam_new"), (v, C, "v"), (dvdl, C, "dvdl"),
                     (ph, R, "ph")):
        _check(t, n, f64, nm)
    _check(partner, C, i32, "partner", True)
    for t, n, nm in ((pka, C, "pka"), (mm, 36 * C, "mm"), (dwp, 4 * C, "dwp"),
                     (noise, 2 * R, "noise"), (stats_w, 5 * C, "stats_w"),
                     (stats_b, 2 * C, "stats_b"), (kin, R, "kin"), (e_bias, R, "e_bias"),
                     (dwp2, 2 * C, "dwp2"), (stats_b2, 2 * C, "stats_b2")):
        _check(t, n, f64, nm, True)
    s = stream if stream is not None else torch.cuda.current_stream(lam.device)
    st = load_library().fmm_lambda_step(
        ctypes.c_void_p(s.cuda_stream), R, _p(coord_off), C, ctypes.byref(params),
        1 if first else 0, _p(lam), _p(lam_new), _p(v), _p(dvdl), _p(partner), _p(pka), _p(ph),
        _p(mm), _p(dwp), _p(noise), _p(stats_w), _p(stats_b), _p(kin), _p(e_bias), _p(dwp2),
        _p(stats_b2))
    _raise(st, "fmm_lambda_step")


def lambda_dbo(coord_off, dwp, ph, temperature, mode=3, pfc=True, pka=None, stats_w=None,
               stats_b=None, adjusted=None, params: DboParams | None = None, stream=None,
               partner=None, dwp2=None, stats_b2=None):
    """fmm_lambda_dbo on device tensors."""
    import torch
    R = coord_off.numel() - 1
    C = dwp.numel() // 4
    _check(coord_off, R + 1, torch.int32, "coord_off")
    _check(dwp, 4 * C, torch.float64, "dwp")
    _check(ph, R, torch.float64, "ph")
    _check(pka, C, torch.float64, "pka", True)
    _check(stats_w, 5 * C, torch.float64, "stats_w", True)
    _check(stats_b, 2 * C, torch.float64, "stats_b", True)
    _check(adjusted, C, torch.int32, "adjusted", True)
    _check(partner, C, torch.int32, "partner", True)
    _check(dwp2, 2 * C, torch.float64, "dwp2", True)
    _check(stats_b2, 2 * C, torch.float64, "stats_b2", True)
    s = stream if stream is not None else torch.cuda.current_stream(dwp.device)
    st = load_library().fmm_lambda_dbo(
        ctypes.c_void_p(s.cuda_stream), R, _p(coord_off), C, int(mode), 1 if pfc else 0,
        ctypes.byref(params) if params is not None else ctypes.c_void_p(0), float(temperature),
        _p(pka), _p(ph), _p(dwp), _p(stats_w), _p(stats_b), _p(adjusted), _p(partner), _p(dwp2),
        _p(stats_b2))
    _raise(st, "fmm_lambda_dbo")


def lambda_pfc(coord_off, dwp, ph, temperature, pka=None, stream=None, partner=None, dwp2=None):
    """fmm_lambda_pfc on device tensors."""
    import torch
    R = coord_off.numel() - 1
    C = dwp.numel() // 4
    _check(coord_off, R + 1, torch.int32, "coord_off")
    _check(dwp, 4 * C, torch.float64, "dwp")
    _check(ph, R, torch.float64, "ph")
    _check(pka, C, torch.float64, "pka", True)
    _check(partner, C, torch.int32, "partner", True)
    _check(dwp2, 2 * C, torch.float64, "dwp2", True)
    s = stream if stream is not None else torch.cuda.current_stream(dwp.device)
    st = load_library().fmm_lambda_pfc(ctypes.c_void_p(s.cuda_stream), R, _p(coord_off), C,
                                       float(temperature), _p(pka), _p(ph), _p(dwp), _p(partner),
                                       _p(dwp2))
    _raise(st, "fmm_lambda_pfc")


class LambdaDynamics:
    """Lambda particles of the sites of R replicas (one coordinate per
    two-form site), advanced by one velocity-Verlet step per Coulomb solve.

    step(dvdl) takes the solve's dV/dlambda per site (kJ/mol: solve with
    coulomb_k = 138.935458) at the current lambda, draws the thermostat's
    random numbers on the device, moves lambda and, every `well_block` /
    `barrier_block` steps, applies DBO (with the partition function
    correction).  The bias parameters default to the paper's barrier of
    6 kJ/mol with wells at 0 and 1 and no V_MM (synthetic: the calibration
    polynomials are inputs, mm).  Tautomer coordinates (pKa NaN with a
    partner) get a second barrier for the deprotonated state, starting at the
    same height and tuned by DBO from its own statistics."""

    def __init__(self, site_off, lam0, ph, pka, mass=60.0, dt=0.002, temperature=300.0,
                 tau=1.0, barrier=6.0, mm=None, partner=None, well_block=None,
                 barrier_block=None, seed=0, device="cuda"):
        import numpy as np
        import torch
        self.dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=self.dev)
        site_off = np.asarray(site_off, dtype=np.int64)
        self.R = site_off.size - 1
        self.C = int(site_off[-1])
        self.coord_off = torch.tensor(site_off, dtype=torch.int32, device=self.dev)
        self.nf = torch.tensor(np.diff(site_off), **f64)
        self.lam = torch.tensor(np.asarray(lam0, dtype=np.float64), **f64)
        self.lam_next = torch.empty_like(self.lam)
        self.ph = torch.tensor(np.asarray(ph, dtype=np.float64), **f64)
        self.pka = torch.tensor(np.asarray(pka, dtype=np.float64), **f64)
        self.mm = None if mm is None else torch.tensor(np.asarray(mm, dtype=np.float64), **f64)
        self.partner = None if partner is None else torch.tensor(np.asarray(partner), dtype=torch.int32,
                                                                 device=self.dev)
        dwp = np.zeros((self.C, 4))
        dwp[:, 0], dwp[:, 2] = barrier, 1.0
        self.dwp = torch.tensor(dwp, **f64)
        taut = (partner is not None and np.any((np.asarray(partner) >= 0)
                                               & np.isnan(np.asarray(pka, dtype=np.float64))))
        # second barrier and y1 of tautomer coordinates (others ignore them)
        self.dwp2 = torch.tensor(np.stack([np.full(self.C, barrier), np.zeros(self.C)], axis=1),
                                 **f64) if taut else None
        self.stats_b2 = torch.zeros(2 * self.C, **f64) if taut else None
        self.params = LambdaParams(mass, dt, temperature, tau, 0.2, 0.8)
        self.T = temperature
        self.gen = torch.Generator(device=self.dev)
        self.gen.manual_seed(seed)
        # initial velocities from the Maxwell distribution at T
        sd = math.sqrt(KB * temperature / mass)
        self.v = torch.randn(self.C, generator=self.gen, **f64) * sd
        self.stats_w = torch.zeros(5 * self.C, **f64)
        self.stats_b = torch.zeros(2 * self.C, **f64)
        self.adjusted = torch.zeros(self.C, dtype=torch.int32, device=self.dev)
        self.kin = torch.zeros(self.R, **f64)
        self.e_bias = torch.zeros(self.R, **f64)
        # thermostat random numbers, drawn for noise_block steps at a time
        self.noise_block = 1000
        self.noise_bank = torch.zeros((self.noise_block, 2 * self.R), **f64)
        self.noise = self.noise_bank[0]
        # wells: 40 ps blocks, barrier: 1 ns blocks ("Dynamic Barrier and Well Optimization")
        self.well_block = well_block if well_block is not None else int(round(40.0 / dt))
        self.barrier_block = barrier_block if barrier_block is not None else int(round(1000.0 / dt))
        self.n = 0
        self._checked = None  # the tensors (and their metadata) the last full check saw
        lambda_pfc(self.coord_off, self.dwp, self.ph, temperature, pka=self.pka,
                   partner=self.partner if self.dwp2 is not None else None, dwp2=self.dwp2)

    def draw_noise(self):
        """For each of the next noise_block steps, one standard normal and one
        chi-square sample with N_f - 1 degrees of freedom per replica: by its
        definition, the sum of N_f - 1 squared standard normals (0 for none),
        drawn in chunks of 256 degrees of freedom."""
        import torch
        nb, R = self.noise_block, self.R
        f64 = dict(dtype=torch.float64, device=self.dev)
        r1 = torch.randn((nb, R), generator=self.gen, **f64)
        k = torch.clamp(self.nf - 1, min=0).reshape(R)
        chi2 = torch.zeros((nb, R), **f64)
        kmax = int(k.max().item()) if R else 0
        for k0 in range(0, kmax, 256):
            w = min(256, kmax - k0)
            z = torch.randn((nb, R, w), generator=self.gen, **f64)
            used = (k0 + torch.arange(w, device=self.dev))[None, :] < k[:, None]
            chi2 += (z * z * used).sum(-1)
        bank = self.noise_bank.view(nb, R, 2)
        bank[:, :, 0] = r1
        bank[:, :, 1] = chi2

    @staticmethod
    def _meta(t):
        return None if t is None else (t.data_ptr(), t.numel(), t.dtype, t.device)

    def _fingerprint(self):
        ts = (self.coord_off, self.v, self.ph, self.partner, self.pka, self.mm, self.dwp,
              self.noise_bank, self.stats_w, self.stats_b, self.kin, self.e_bias,
              getattr(self, "dwp2", None), getattr(self, "stats_b2", None))
        return ([(t, self._meta(t)) for t in ts],
                sorted([(self.lam, self._meta(self.lam)), (self.lam_next, self._meta(self.lam_next))],
                       key=lambda e: e[1][0]))

    @staticmethod
    def _same(a, b):
        """Same tensor objects (compared with `is`) with unchanged metadata."""
        if a is None or b is None:
            return False
        pa = a[0] + a[1]
        pb = b[0] + b[1]
        return len(pa) == len(pb) and all(x[0] is y[0] and x[1] == y[1] for x, y in zip(pa, pb))

    def step(self, dvdl):
        if self.params.tau > 0:
            i = self.n % self.noise_block
            if i == 0:
                self.draw_noise()
            self.noise = self.noise_bank[i]
        # the full tensor checks run again whenever a tensor was replaced or
        # changed in place (lam and lam_next alternate; the noise row moves
        # through one bank; dvdl, usually a fresh tensor per solve, is checked
        # on every call): the last checked tensors are kept (so their
        # identities cannot be reused) with their storage, size, type and device
        seen = self._fingerprint()
        lambda_step(self.coord_off, self.lam, self.lam_next, self.v, dvdl, self.ph, self.params,
                    first=self.n == 0, partner=self.partner, pka=self.pka, mm=self.mm,
                    dwp=self.dwp, noise=self.noise if self.params.tau > 0 else None,
                    stats_w=self.stats_w, stats_b=self.stats_b, kin=self.kin, e_bias=self.e_bias,
                    check=not self._same(seen, self._checked), dwp2=self.dwp2,
                    stats_b2=self.stats_b2)
        self._checked = seen
        self.lam, self.lam_next = self.lam_next, self.lam
        self.n += 1
        mode = (1 if self.n % self.well_block == 0 else 0) | (2 if self.n % self.barrier_block == 0 else 0)
        if mode:
            lambda_dbo(self.coord_off, self.dwp, self.ph, self.T, mode=mode, pfc=True,
                       pka=self.pka, stats_w=self.stats_w, stats_b=self.stats_b,
                       adjusted=self.adjusted,
                       partner=self.partner if self.dwp2 is not None else None,
                       dwp2=self.dwp2, stats_b2=self.stats_b2)
        return self.lam
