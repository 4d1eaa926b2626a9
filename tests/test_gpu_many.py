"""Many signals through one prepared kernel in one launch (apx_many_*), against the oracle.

Every signal's output equals the oracle's (packed modes bit for bit, FP32 within the FP32 bound)
and equals the single-signal run (apx_run) bit for bit, on the time-domain, integer and FFT
cores, for signals of uneven length (one block, ragged tails, the shortest admissible length).
The time-domain workload (1024 signals of 65536 samples, asymmetric packing at 8 bits) is
checked in full against the single-signal runs and on sampled signals against the oracle.
"""
import numpy as np
import pytest

import oracle as O
from paper_1201_3018_amd import synth
from gpu_checks import check_mixed_blocks, fp32_bound

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1201_3018_amd import apx  # noqa: E402

DEV = torch.device("cuda:0")
MODES = {O.SYM: apx.APX_SYM, O.ASYM2: apx.APX_ASYM2, O.ASYM3: apx.APX_ASYM3}


@pytest.fixture(scope="module")
def ctx():
    c = apx.Context(0)
    yield c
    c.close()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def _say(*a):
    print(*a, flush=True)


def _lengths(N, Wb, seed, n=7):
    No = N if N % 2 else N + 1
    W = Wb - No - 1
    rng = np.random.default_rng(seed)
    Ls = [N, W, W + 1, 3 * W - 2, 5 * W + 777] + [int(x) for x in rng.integers(N, 12 * W, n - 5)]
    return Ls


CASES = [  # (core, variant, mode, N, W_block)
    ("td", apx.FFT_AUTO, O.SYM, 64, 1024),
    ("td", apx.FFT_AUTO, O.ASYM2, 101, 1024),
    ("td", apx.FFT_AUTO, "fp32", 64, 1024),
    ("int8", apx.FFT_AUTO, O.ASYM2, 64, 1024),
    ("int8", apx.FFT_AUTO, O.SYM, 129, 2048),
    ("fft", apx.FFT_WAVE, O.ASYM2, 1024, 4096),
    ("fft", apx.FFT_GROUP, O.ASYM2, 1024, 4096),
    ("fft", apx.FFT_GROUP, O.SYM, 1024, 4096),
    ("fft", apx.FFT_BLOCK, O.ASYM3, 300, 2048),
    ("fft", apx.FFT_GROUP, "fp32", 1024, 4096),
]
CORES = {"td": apx.APX_CORE_TIME, "fft": apx.APX_CORE_FFT, "int8": apx.APX_CORE_INT8}


@pytest.mark.parametrize("core,variant,mode,N,Wb", CASES)
def test_many_equals_oracle_and_single(ctx, core, variant, mode, N, Wb):
    No = N if N % 2 else N + 1
    Ls = _lengths(N, Wb, 900 + N)
    _say("case: many", core, variant, mode, N, Wb, "lengths", Ls)
    sigs = [synth.ar1(L, 910 + i) for i, L in enumerate(Ls)]
    k = synth.hann_lowpass(N, 0.15)
    am = apx.APX_FULL_FP32 if mode == "fp32" else MODES[mode]
    S = 0 if mode == "fp32" else O.max_q(mode, No)
    kern = apx.Kernel(ctx, _dev(k), Wb, mode=am, core=CORES[core], Sq=S, Kq=S, fft_variant=variant)
    ts = [_dev(x) for x in sigs]
    outs0 = [torch.full((x.numel() + N - 1,), float("nan"), dtype=torch.float32, device=DEV) for x in ts]
    many = apx.Many(kern, ts, outs=outs0, info=True)
    _say(" ", many.describe())
    outs = many.run()
    torch.cuda.synchronize()
    for i, (x, t) in enumerate(zip(sigs, ts)):
        got = outs[i].cpu().numpy()
        single = torch.full_like(outs[i], float("nan"))
        single, sinfo = kern.run(t, out=single, info=True)
        torch.cuda.synchronize()
        assert np.array_equal(got.view(np.int32), single.cpu().numpy().view(np.int32)), i
        assert np.array_equal(apx.block_info(many.infos[i]), apx.block_info(sinfo)), i
        if mode == "fp32":
            err = np.abs(got.astype(np.float64) - O.conv_direct(x, k))
            assert np.all(err <= fp32_bound(x, k, Wb, core)), (i, float(np.max(err)))
        else:
            ref = O.conv_blocked(x, k, Wb, O.fixed_params(x, k, Wb, mode, S, S))
            assert np.array_equal(got.view(np.int32), ref.view(np.int32)), (i, int(np.sum(got != ref)))
    many.close()
    kern.close()


def test_many_auto_snr_mixed_modes(ctx):
    """APX_AUTO_SNR with the kernel's calibration: signals whose blocks choose different modes
    (symmetric, asymmetric M=2, FP32) in one launch; packed blocks bit for bit, FP32 blocks in
    the bound, and equal to the single runs."""
    N, Wb, target = 1024, 4096, 38.0
    Ls = _lengths(N, Wb, 77)
    sigs = [synth.ar1(L, 960 + i) * np.float32(1.0 + 0.5 * i) for i, L in enumerate(Ls)]
    sigs[2] = synth.gaussian(Ls[2], 5)  # a white signal: other model SNRs
    k = synth.hann_lowpass(N)
    calib = O.calibrate(sigs[-1], k, Wb)
    kern = apx.Kernel(ctx, _dev(k), Wb, mode=apx.APX_AUTO_SNR, core=apx.APX_CORE_FFT, snr_min_db=target,
                      calib_db=calib)
    ts = [_dev(x) for x in sigs]
    outs0 = [torch.full((x.numel() + N - 1,), float("nan"), dtype=torch.float32, device=DEV) for x in ts]
    many = apx.Many(kern, ts, outs=outs0, info=True)
    outs = many.run()
    torch.cuda.synchronize()
    counts = np.zeros(3, np.int64)
    for i, (x, t) in enumerate(zip(sigs, ts)):
        got = outs[i].cpu().numpy()
        info = apx.block_info(many.infos[i])
        single = kern.run(t)
        torch.cuda.synchronize()
        assert np.array_equal(got.view(np.int32), single.cpu().numpy().view(np.int32)), i
        ps = O.auto_params(x, k, Wb, target, calib)
        want = np.array([{O.SYM: 1, O.ASYM2: 2, O.FULL: 0}[p.mode] for p in ps])
        near = np.array([abs(p.snr_pred_db - target) < 1e-6 for p in ps])
        assert np.array_equal(info["mode"][~near], want[~near]), i
        check_mixed_blocks(x, k, Wb, ps, info["mode"], got, "fft")
        counts += np.bincount(info["mode"], minlength=3)[:3]
    _say(f"  block modes over all signals (FP32, sym, asym2): {counts}")
    many.close()
    kern.close()


def test_many_time_domain_workload(ctx):
    """1024 signals of 65536 N(0,1) samples, kernel of 64 U(-1,1) taps, W_block 1024, asymmetric
    packing at 8 bits (S_q = K_q = 127), as one launch: every output equals its single-signal run,
    and eight sampled signals equal the oracle."""
    n, L, N, Wb = 1024, 65536, 64, 1024
    k = synth.uniform(N, 1002)
    base = synth.gaussian(L * 8, 1001).reshape(8, L)
    rng = np.random.default_rng(11)
    # 1024 distinct signals from 8 generated rows: sign flips and circular shifts
    host = np.empty((n, L), np.float32)
    for i in range(n):
        host[i] = np.roll(base[i % 8], int(rng.integers(0, L))) * (1.0 if (i // 8) % 2 == 0 else -1.0)
    dev = torch.from_numpy(host).to(DEV)
    kern = apx.Kernel(ctx, _dev(k), Wb, mode=apx.APX_ASYM2, Sq=127, Kq=127)
    _say("  kernel:", kern.describe())
    ts = [dev[i] for i in range(n)]
    many = apx.Many(kern, ts)
    _say(" ", many.describe())
    many.run()
    torch.cuda.synchronize()
    out = torch.stack(many.outs).cpu().numpy()
    single = torch.empty_like(many.outs[0])
    for i in range(n):
        kern.run(ts[i], out=single)
        torch.cuda.synchronize() if i % 256 == 255 else None
        assert torch.equal(single, many.outs[i]), i
    for i in (0, 1, 77, 255, 256, 511, 900, 1023):
        ref = O.conv_blocked(host[i], k, Wb, O.fixed_params(host[i], k, Wb, O.ASYM2, 127, 127))
        assert np.array_equal(out[i].view(np.int32), ref.view(np.int32)), i
    snr = O.measured_snr_db(out[0], O.conv_direct(host[0], k))
    _say(f"  SNR of signal 0 against FP64: {snr:.2f} dB")
    assert snr >= 40.0
    many.close()
    kern.close()


def test_many_errors(ctx):
    k = _dev(synth.uniform(64, 3))
    kern = apx.Kernel(ctx, k, 1024, mode=apx.APX_SYM)
    s = _dev(synth.gaussian(5000, 4))
    with pytest.raises(apx.ApxError) as e:
        apx.Many(kern, [s, _dev(np.zeros(10, np.float32))])      # shorter than the kernel
    assert e.value.status == apx.APX_E_INVALID
    buf = torch.zeros(5001, dtype=torch.float32, device=DEV)
    with pytest.raises(apx.ApxError) as e:
        apx.Many(kern, [s, buf[1:]])                              # misaligned
    assert e.value.status == apx.APX_E_INVALID
    with pytest.raises(apx.ApxError) as e:
        apx.Many(kern, [])
    assert e.value.status == apx.APX_E_INVALID
    kern.close()
