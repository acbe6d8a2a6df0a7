"""Host-side argument checks of the lambda-dynamics calls: invalid arguments
are rejected before anything is enqueued (no GPU needed)."""
import ctypes

from paper_2410_01626_amd import fmm
from paper_2410_01626_amd import lambda_dynamics as LD

NULL = ctypes.c_void_p(0)
FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def _step(R=1, C=4, prm=None, first=0, lam=FAKE, lam_new=ctypes.c_void_p(0x2000), noise=NULL,
          coord_off=FAKE, ph=FAKE):
    lib = fmm.load_library()
    prm = prm if prm is not None else LD.LambdaParams(60.0, 0.002, 300.0, 0.0, 0.2, 0.8)
    return lib.fmm_lambda_step(NULL, R, coord_off, C, ctypes.byref(prm), first, lam, lam_new,
                               FAKE, FAKE, NULL, NULL, ph, NULL, NULL, noise, NULL, NULL, NULL, NULL)


def test_lambda_step_rejects_bad_arguments():
    bad = [dict(R=0), dict(C=-1), dict(first=2), dict(coord_off=NULL), dict(ph=NULL),
           dict(lam=NULL), dict(lam_new=FAKE),  # aliasing the input
           dict(prm=LD.LambdaParams(0.0, 0.002, 300.0, 0.0, 0.2, 0.8)),
           dict(prm=LD.LambdaParams(60.0, -1.0, 300.0, 0.0, 0.2, 0.8)),
           dict(prm=LD.LambdaParams(60.0, 0.002, float("nan"), 0.0, 0.2, 0.8)),
           dict(prm=LD.LambdaParams(60.0, 0.002, 300.0, 0.0, 0.9, 0.1)),
           dict(prm=LD.LambdaParams(60.0, 0.002, 300.0, 1.0, 0.2, 0.8))]  # thermostat, no noise
    for kw in bad:
        assert _step(**kw) == fmm.FMM_E_INVALID, kw


def test_lambda_dbo_and_pfc_reject_bad_arguments():
    lib = fmm.load_library()
    args = lambda R=1, C=4, mode=3, pfc=1, T=300.0, dwp=FAKE, sw=FAKE, sb=FAKE: (
        NULL, R, FAKE, C, mode, pfc, NULL, T, NULL, FAKE, dwp, sw, sb, NULL)
    for kw in (dict(R=0), dict(mode=4), dict(mode=-1), dict(pfc=2), dict(T=0.0), dict(dwp=NULL),
               dict(mode=1, sw=NULL), dict(mode=2, sb=NULL)):
        assert lib.fmm_lambda_dbo(*args(**kw)) == fmm.FMM_E_INVALID, kw
    assert lib.fmm_lambda_pfc(NULL, 1, FAKE, 4, -1.0, NULL, FAKE, FAKE) == fmm.FMM_E_INVALID
    assert lib.fmm_lambda_pfc(NULL, 1, FAKE, 4, 300.0, NULL, FAKE, NULL) == fmm.FMM_E_INVALID
    assert lib.fmm_lambda_pfc(NULL, 1, NULL, 4, 300.0, NULL, FAKE, FAKE) == fmm.FMM_E_INVALID


def test_param_struct_layouts():
    assert ctypes.sizeof(LD.LambdaParams) == 48
    assert ctypes.sizeof(LD.DboParams) == 88
