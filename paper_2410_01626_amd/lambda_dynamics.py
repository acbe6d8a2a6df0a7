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
                stats_b=None, kin=None, e_bias=None, stream=None, check=True):
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
            _p(mm), _p(dwp), _p(noise), _p(stats_w), _p(stats_b), _p(kin), _p(e_bias))
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
                     (stats_b, 2 * C, "stats_b"), (kin, R, "kin"), (e_bias, R, "e_bias")):
        _check(t, n, f64, nm, True)
    s = stream if stream is not None else torch.cuda.current_stream(lam.device)
    st = load_library().fmm_lambda_step(
        ctypes.c_void_p(s.cuda_stream), R, _p(coord_off), C, ctypes.byref(params),
        1 if first else 0, _p(lam), _p(lam_new), _p(v), _p(dvdl), _p(partner), _p(pka), _p(ph),
        _p(mm), _p(dwp), _p(noise), _p(stats_w), _p(stats_b), _p(kin), _p(e_bias))
    _raise(st, "fmm_lambda_step")


def lambda_dbo(coord_off, dwp, ph, temperature, mode=3, pfc=True, pka=None, stats_w=None,
               stats_b=None, adjusted=None, params: DboParams | None = None, stream=None):
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
    s = stream if stream is not None else torch.cuda.current_stream(dwp.device)
    st = load_library().fmm_lambda_dbo(
        ctypes.c_void_p(s.cuda_stream), R, _p(coord_off), C, int(mode), 1 if pfc else 0,
        ctypes.byref(params) if params is not None else ctypes.c_void_p(0), float(temperature),
        _p(pka), _p(ph), _p(dwp), _p(stats_w), _p(stats_b), _p(adjusted))
    _raise(st, "fmm_lambda_dbo")


def lambda_pfc(coord_off, dwp, ph, temperature, pka=None, stream=None):
    """fmm_lambda_pfc on device tensors."""
    import torch
    R = coord_off.numel() - 1
    C = dwp.numel() // 4
    _check(coord_off, R + 1, torch.int32, "coord_off")
    _check(dwp, 4 * C, torch.float64, "dwp")
    _check(ph, R, torch.float64, "ph")
    _check(pka, C, torch.float64, "pka", True)
    s = stream if stream is not None else torch.cuda.current_stream(dwp.device)
    st = load_library().fmm_lambda_pfc(ctypes.c_void_p(s.cuda_stream), R, _p(coord_off), C,
                                       float(temperature), _p(pka), _p(ph), _p(dwp))
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
    polynomials are inputs, mm)."""

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
        self._checked = None  # identities of the tensors the last full check saw
        lambda_pfc(self.coord_off, self.dwp, self.ph, temperature, pka=self.pka)

    def draw_noise(self):
        """For each of the next noise_block steps, one standard normal and one
        chi-square sample with N_f - 1 degrees of freedom per replica
        (chi^2_k = 2 Gamma(k / 2, 1); 0 for k = 0)."""
        import torch
        nb, R = self.noise_block, self.R
        r1 = torch.randn((nb, R), generator=self.gen, dtype=torch.float64, device=self.dev)
        k = torch.clamp(self.nf - 1, min=0).expand(nb, R).contiguous()
        g = torch._standard_gamma(torch.clamp(k / 2, min=1e-300), generator=self.gen)
        chi2 = torch.where(k > 0, 2 * g, torch.zeros_like(g))
        bank = self.noise_bank.view(nb, R, 2)
        bank[:, :, 0] = r1
        bank[:, :, 1] = chi2

    def step(self, dvdl):
        if self.params.tau > 0:
            i = self.n % self.noise_block
            if i == 0:
                self.draw_noise()
            self.noise = self.noise_bank[i]
        # the full tensor checks run again whenever a tensor was replaced
        # (lam and lam_next alternate; the noise row moves through one bank)
        # (dvdl, usually a fresh tensor per solve, is checked on every call)
        seen = tuple(id(t) for t in (self.coord_off, self.v, self.ph, self.partner, self.pka,
                                     self.mm, self.dwp, self.noise_bank, self.stats_w,
                                     self.stats_b, self.kin, self.e_bias)) + (
            frozenset((id(self.lam), id(self.lam_next))),)
        lambda_step(self.coord_off, self.lam, self.lam_next, self.v, dvdl, self.ph, self.params,
                    first=self.n == 0, partner=self.partner, pka=self.pka, mm=self.mm,
                    dwp=self.dwp, noise=self.noise if self.params.tau > 0 else None,
                    stats_w=self.stats_w, stats_b=self.stats_b, kin=self.kin, e_bias=self.e_bias,
                    check=seen != self._checked)
        self._checked = seen
        self.lam, self.lam_next = self.lam_next, self.lam
        self.n += 1
        mode = (1 if self.n % self.well_block == 0 else 0) | (2 if self.n % self.barrier_block == 0 else 0)
        if mode:
            lambda_dbo(self.coord_off, self.dwp, self.ph, self.T, mode=mode, pfc=True,
                       pka=self.pka, stats_w=self.stats_w, stats_b=self.stats_b,
                       adjusted=self.adjusted)
        return self.lam
