"""Marginal-CDF modelling on the device (Section IV.D, Fig. 4) against the oracle.

apx_fit_marginal: the zero-mean Laplacian and two-parameter Weibull maximum-likelihood fits equal
the oracle's to 1e-10 relative (same equations, different summation order).
Source-level sigmas (apx_params.sigma_s / sigma_k) in eq. (18): per-block modes equal the
oracle's selection except at exact ties, packed blocks bit-exact, the reported model SNR equal
to the oracle's, and calibration (host and device) equal to the oracle's offset.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1201_3018_amd import synth
from gpu_checks import check_mixed_blocks

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1201_3018_amd import apx  # noqa: E402

DEV = torch.device("cuda:0")
MODEL = {O.marginal.LAPLACE: apx.APX_MARGINAL_LAPLACE, O.marginal.WEIBULL: apx.APX_MARGINAL_WEIBULL}


@pytest.fixture(scope="module")
def ctx():
    c = apx.Context(0)
    yield c
    c.close()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def _say(*a):
    print(*a, flush=True)


def _sources():
    rng = np.random.default_rng(8100)
    w = (0.7 * rng.weibull(2.2, 50000)).astype(np.float32)
    w[::97] = 0.0  # zeros: left out of a Weibull fit
    return [("ar1 audio", synth.ar1(1 << 20, 8101), O.marginal.LAPLACE),
            ("gaussian", synth.gaussian(300001, 8102), O.marginal.LAPLACE),
            ("weibull features", synth.weibull_features(1 << 20, 8103), O.marginal.WEIBULL),
            ("weibull iid with zeros", w, O.marginal.WEIBULL),
            ("tiny", np.array([0.5, 2.0, 1.0], np.float32), O.marginal.WEIBULL)]


@pytest.mark.parametrize("case", range(5))
def test_fit_marginal_matches_oracle(ctx, case):
    name, x, model = _sources()[case]
    _say(f"marginal fit {name}: {model}, n={x.size}")
    g = apx.apx_fit_marginal(ctx.h, _dev(x), MODEL[model])
    o = O.marginal.fit(x, model)
    _say(f"  device {g}  oracle {o}")
    assert g[3] == o.n
    for gv, ov in ((g[0], o.scale), (g[1], o.shape), (g[2], o.sigma)):
        assert abs(gv - ov) <= 1e-10 * abs(ov), (gv, ov)


def test_fit_marginal_errors(ctx):
    with pytest.raises(apx.ApxError) as e:
        apx.apx_fit_marginal(ctx.h, _dev(-np.ones(100)), apx.APX_MARGINAL_WEIBULL)
    assert e.value.status == apx.APX_E_INVALID
    with pytest.raises(apx.ApxError) as e:
        apx.apx_fit_marginal(ctx.h, _dev(np.ones(100)), 7)
    assert e.value.status == apx.APX_E_INVALID


def _check_auto(s, k, Wb, target, calib, sigma_s, sigma_k, got, info):
    kmax, krms = O.kernel_stats(k)
    ps = O.marginal.auto_params_sigma(s, k, Wb, target, sigma_s, sigma_k or krms, calib)
    want = np.array([{O.SYM: 1, O.ASYM2: 2, O.FULL: 0}[p.mode] for p in ps])
    near = np.array([abs(p.snr_pred_db - target) < 1e-6 for p in ps])
    assert np.array_equal(info["mode"][~near], want[~near])
    packed = (info["mode"] != 0) & ~near & np.isfinite([p.snr_pred_db for p in ps])
    pred = np.array([p.snr_pred_db for p in ps])
    assert np.allclose(info["snr_pred_db"][packed], pred[packed], rtol=0, atol=1e-9)
    check_mixed_blocks(s, k, Wb, ps, info["mode"], got, "fft")
    return np.bincount(info["mode"], minlength=3)


@pytest.mark.parametrize("N,Wb,core", [(1024, 4096, apx.APX_CORE_FFT), (65, 1024, apx.APX_CORE_TIME),
                                       (300, 2048, apx.APX_CORE_FFT), (1000, 8192, apx.APX_CORE_FFT),
                                       (2000, 16384, apx.APX_CORE_FFT)])
@pytest.mark.parametrize("split", [O.SYM, O.ASYM2])
def test_source_sigma_selection(ctx, N, Wb, core, split):
    """AUTO selection with the signal's Laplacian sigma and the taps' Laplacian sigma, at the
    target that splits the blocks' model SNR of one packing in half (a mix of modes)."""
    s = synth.ar1(200000, 8200 + N)
    k = synth.hann_lowpass(N, 0.1)
    ts = _dev(s)
    sig_s = apx.apx_fit_marginal(ctx.h, ts, apx.APX_MARGINAL_LAPLACE)[2]
    sig_k = apx.apx_fit_marginal(ctx.h, _dev(k), apx.APX_MARGINAL_LAPLACE)[2]
    calib = 3.25
    part = O.partition(len(s), len(k), Wb)
    kmax, _ = O.kernel_stats(k)
    q = O.max_q(split, part.N_odd)
    model = [O.snr_model_db(sig_s, O.block_stats(part.window(s, w))[0], sig_k, kmax, q, q) + calib
             for w in range(part.P)]
    target = float(np.median(model)) + 1e-3
    kern = apx.Kernel(ctx, _dev(k), Wb, mode=apx.APX_AUTO_SNR, core=core, snr_min_db=target, calib_db=calib,
                      sigma_s=sig_s, sigma_k=sig_k)
    out, info = kern.run(ts, info=True)
    torch.cuda.synchronize()
    got, info = out.cpu().numpy(), apx.block_info(info)
    _say(f"source sigmas N={N}: sigma_s={sig_s:.6f} sigma_k={sig_k:.6f} ({kern.describe()[:40]})")
    kern.close()
    counts = _check_auto(s, k, Wb, target, calib, sig_s, sig_k, got, info)
    _say(f"  modes {counts}")


def test_source_sigma_fixed_mode_report_and_calibration(ctx):
    s = synth.ar1(100000, 8301)
    k = synth.hann_lowpass(257, 0.15)
    Wb = 2048
    ts, tk = _dev(s), _dev(k)
    sig_s = 0.123456
    kmax, krms = O.kernel_stats(k)
    S = O.max_q(O.ASYM2, 257)
    kern = apx.Kernel(ctx, tk, Wb, mode=apx.APX_ASYM2, core=apx.APX_CORE_FFT, Sq=S, Kq=S, sigma_s=sig_s)
    _, info = kern.run(ts, info=True)
    torch.cuda.synchronize()
    info = apx.block_info(info)
    kern.close()
    want = np.array([O.snr_model_db(sig_s, smax, krms, kmax, S, S) for smax in info["smax"]])
    assert np.allclose(info["snr_pred_db"], want, rtol=0, atol=1e-9)
    # calibration at Q = 8 on block 1: the measured SNR minus the model with the source sigma
    part = O.partition(len(s), len(k), Wb)
    smax1, rms1 = O.block_stats(part.window(s, 1))
    measured = O.calibrate(s, k, Wb, block=1, Q=8) + O.snr_model_db(rms1, smax1, krms, kmax, 8, 8)
    expect = measured - O.snr_model_db(sig_s, smax1, krms, kmax, 8, 8)
    kauto = apx.Kernel(ctx, tk, Wb, mode=apx.APX_AUTO_SNR, core=apx.APX_CORE_FFT, snr_min_db=40.0, sigma_s=sig_s)
    off = apx.apx_calibrate(ctx.h, kauto.h, ts, block=1, Q=8)
    assert abs(off - expect) < 1e-6, (off, expect)
    # the per-call device calibration of apx_run_auto lands on the same offset and selection
    ws = torch.empty(apx.apx_workspace_bytes(), dtype=torch.uint8, device=DEV)
    out = torch.empty(len(s) + len(k) - 1, dtype=torch.float32, device=DEV)
    inf = torch.empty(part.P * apx.BLOCK_INFO_DTYPE.itemsize, dtype=torch.uint8, device=DEV)
    apx.apx_run_auto(ctx.h, kauto.h, ts, out, 40.0, 1, ws, inf)
    torch.cuda.synchronize()
    kauto.close()
    _check_auto(s, k, Wb, 40.0, expect, sig_s, 0.0, out.cpu().numpy(), apx.block_info(inf))
    assert not math.isnan(off)
