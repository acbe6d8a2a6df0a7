"""Host-side argument checks of the lambda-dynamics calls: invalid arguments
are rejected before anything is enqueued (no GPU needed)."""
import ctypes

from paper_2410_01626_amd import fmm
from paper_2410_01626_amd import lambda_dynamics as LD

NULL = ctypes.c_void_p(0)
FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def _step(R=1, C=4, prm=None, first=0, lam=FAKE, lam_new=ctypes.c_void_p(0x2000), noise=NULL,
          coord_off=FAKE, ph=FAKE, partner=NULL, dwp=NULL, stats_b=NULL, dwp2=NULL, stats_b2=NULL):
    lib = fmm.load_library()
    prm = prm if prm is not None else LD.LambdaParams(60.0, 0.002, 300.0, 0.0, 0.2, 0.8)
    return lib.fmm_lambda_step(NULL, R, coord_off, C, ctypes.byref(prm), first, lam, lam_new,
                               FAKE, FAKE, partner, NULL, ph, NULL, dwp, noise, NULL, stats_b, NULL,
                               NULL, dwp2, stats_b2)


def test_lambda_step_rejects_bad_arguments():
    bad = [dict(R=0), dict(C=-1), dict(first=2), dict(coord_off=NULL), dict(ph=NULL),
           dict(lam=NULL), dict(lam_new=FAKE),  # aliasing the input
           dict(prm=LD.LambdaParams(0.0, 0.002, 300.0, 0.0, 0.2, 0.8)),
           dict(prm=LD.LambdaParams(60.0, -1.0, 300.0, 0.0, 0.2, 0.8)),
           dict(prm=LD.LambdaParams(60.0, 0.002, float("nan"), 0.0, 0.2, 0.8)),
           dict(prm=LD.LambdaParams(60.0, 0.002, 300.0, 0.0, 0.9, 0.1)),
           dict(prm=LD.LambdaParams(60.0, 0.002, 300.0, 1.0, 0.2, 0.8)),  # thermostat, no noise
           dict(dwp2=FAKE, partner=FAKE),  # second barriers without dwp
           dict(dwp2=FAKE, dwp=FAKE),      # ... or without partners
           dict(stats_b2=FAKE, stats_b=FAKE, dwp=FAKE, partner=FAKE)]  # split stats, no dwp2
    for kw in bad:
        assert _step(**kw) == fmm.FMM_E_INVALID, kw


def test_lambda_dbo_and_pfc_reject_bad_arguments():
    lib = fmm.load_library()
    args = lambda R=1, C=4, mode=3, pfc=1, T=300.0, dwp=FAKE, sw=FAKE, sb=FAKE, partner=NULL, \
        dwp2=NULL, sb2=NULL: (NULL, R, FAKE, C, mode, pfc, NULL, T, NULL, FAKE, dwp, sw, sb, NULL,
                              partner, dwp2, sb2)
    for kw in (dict(R=0), dict(mode=4), dict(mode=-1), dict(pfc=2), dict(T=0.0), dict(dwp=NULL),
               dict(mode=1, sw=NULL), dict(mode=2, sb=NULL),
               dict(dwp2=FAKE, sb2=FAKE),  # second barriers without partners
               dict(mode=2, dwp2=FAKE, partner=FAKE)):  # barrier rule without stats_b2
        assert lib.fmm_lambda_dbo(*args(**kw)) == fmm.FMM_E_INVALID, kw
    assert lib.fmm_lambda_pfc(NULL, 1, FAKE, 4, -1.0, NULL, FAKE, FAKE, NULL, NULL) == fmm.FMM_E_INVALID
    assert lib.fmm_lambda_pfc(NULL, 1, FAKE, 4, 300.0, NULL, FAKE, NULL, NULL, NULL) == fmm.FMM_E_INVALID
    assert lib.fmm_lambda_pfc(NULL, 1, NULL, 4, 300.0, NULL, FAKE, FAKE, NULL, NULL) == fmm.FMM_E_INVALID
    assert lib.fmm_lambda_pfc(NULL, 1, FAKE, 4, 300.0, NULL, FAKE, FAKE, NULL, FAKE) == fmm.FMM_E_INVALID


def test_param_struct_layouts():
    assert ctypes.sizeof(LD.LambdaParams) == 48
    assert ctypes.sizeof(LD.DboParams) == 88


def test_driver_recheck_fingerprint():
    """The driver's skip-the-checks test holds the tensors it saw: a replaced
    tensor (even one that could reuse a freed object's identity), a resize in
    place or a new dtype triggers the full checks again; swapping lam and
    lam_next does not."""
    import torch
    d = LD.LambdaDynamics.__new__(LD.LambdaDynamics)
    names = ("coord_off", "v", "ph", "partner", "pka", "mm", "dwp", "noise_bank", "stats_w",
             "stats_b", "kin", "e_bias", "lam", "lam_next")
    for k in names:
        setattr(d, k, torch.zeros(4, dtype=torch.float64))
    d.partner = None
    a = d._fingerprint()
    assert d._same(a, d._fingerprint())
    d.lam, d.lam_next = d.lam_next, d.lam
    assert d._same(a, d._fingerprint())
    d.v = torch.zeros(4, dtype=torch.float64)  # replaced
    assert not d._same(a, d._fingerprint())
    b = d._fingerprint()
    d.v.resize_(8)  # resized in place
    assert not d._same(b, d._fingerprint())
    c = d._fingerprint()
    d.kin = d.kin.to(torch.float32)
    assert not d._same(c, d._fingerprint())
    assert not d._same(None, d._fingerprint())
