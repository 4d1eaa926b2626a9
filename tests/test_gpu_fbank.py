"""Filter bank on split-precision matrix cores (apx_fbank_*) against the FP64 oracle.

Bound per output (x and h split into high and low half-precision parts, three products, FP32
accumulation over the padded tap count K):
    |y - y64| <= (3 e + (K + 2) 2^-24) (|x| * |h|)[t] + a (sum|x_window| + sum|h|),
    e = 2^-22 (FP16 parts), 2^-16 (BF16 parts)
(e covers the dropped lo*lo product and the rounding of the low parts; the second term the
FP32 accumulation; a = 2^-35 covers FP16 subnormals: a value below 2^-14 keeps an absolute
residual of at most 2^-37 after its two parts, a = 0 for BF16).  The per-channel SNR against
FP64 is printed.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1201_3018_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1201_3018_amd import apx  # noqa: E402

DEV = torch.device("cuda:0")
EPS = {apx.APX_FB_F16X3: 2.0 ** -22, apx.APX_FB_BF16X3: 2.0 ** -16}
ABS = {apx.APX_FB_F16X3: 2.0 ** -35, apx.APX_FB_BF16X3: 0.0}
NAME = {apx.APX_FB_F16X3: "f16x3", apx.APX_FB_BF16X3: "bf16x3"}


@pytest.fixture(scope="module")
def ctx():
    c = apx.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)


def _kpad(N):
    return 128 if N <= 128 else (256 if N <= 256 else 512)


def _check_bank(x, h, y, prec, L):
    C, F, N = x.shape[0], h.shape[0], h.shape[1]
    K = _kpad(N)
    coef = 3 * EPS[prec] + (K + 2) * 2.0 ** -24
    worst = 0.0
    for c in range(C):
        num = den = 0.0
        for f in range(F):
            ref = O.conv_direct(x[c, :L], h[f])
            ax, ah = np.abs(x[c, :L].astype(np.float64)), np.abs(h[f].astype(np.float64))
            bound = coef * O.conv_direct(ax, ah) + ABS[prec] * (O.conv_direct(ax, np.ones(N)) + float(np.sum(ah)))
            got = y[c, f, :L + N - 1].astype(np.float64)
            err = np.abs(got - ref)
            bad = np.nonzero(err > bound + 1e-30)[0]
            assert bad.size == 0, f"c={c} f={f}: {bad.size} outputs beyond the bound, first {bad[:5]}"
            num += float(np.sum(ref * ref))
            den += float(np.sum(err * err))
            worst = max(worst, float(np.max(err / (bound + 1e-30))))
        snr = math.inf if den == 0 else 10 * math.log10(num / den)
        _say(f"  {NAME[prec]} channel {c}: SNR vs FP64 {snr:.1f} dB")
    return worst


@pytest.mark.parametrize("prec", [apx.APX_FB_F16X3, apx.APX_FB_BF16X3])
@pytest.mark.parametrize("C,L,F,N", [(3, 5000, 5, 37), (2, 3000, 32, 512), (1, 100, 1, 1), (2, 1030, 7, 128),
                                     (1, 2500, 32, 129), (1, 700, 3, 300), (1, 40, 2, 64)])
def test_fbank_small(ctx, prec, C, L, F, N):
    rng = np.random.default_rng(1000 * C + N + F)
    x = synth.pink_noise(C, L, 4100 + N) if L >= 16 else rng.standard_normal((C, L)).astype(np.float32)
    h = rng.uniform(-1, 1, (F, N)).astype(np.float32)
    _say(f"fbank {NAME[prec]} C={C} L={L} F={F} N={N}")
    fb = apx.FilterBank(ctx, torch.from_numpy(h).to(DEV), prec)
    y = fb.run(torch.from_numpy(x).to(DEV))
    torch.cuda.synchronize()
    w = _check_bank(x, h, y.cpu().numpy(), prec, L)
    _say(f"  worst error / bound = {w:.3g}")
    fb.close()


def test_fbank_strides_and_errors(ctx):
    rng = np.random.default_rng(5)
    C, L, F, N = 2, 4000, 4, 60
    x = rng.standard_normal((C, L + 13)).astype(np.float32)   # ldx > L
    h = rng.uniform(-1, 1, (F, N)).astype(np.float32)
    fb = apx.FilterBank(ctx, torch.from_numpy(h).to(DEV), apx.APX_FB_F16X3)
    ldy = L + N - 1 + 5                                        # ldy > L + N - 1, not a multiple of 4
    y = torch.full((C * F, ldy), 7.0, device=DEV)
    fb.run(torch.from_numpy(x).to(DEV), y=y, L=L)
    torch.cuda.synchronize()
    yc = y.view(C, F, ldy).cpu().numpy()
    assert np.all(yc[:, :, L + N - 1:] == 7.0)                # padding untouched
    _check_bank(x[:, :L], h, yc, apx.APX_FB_F16X3, L)
    # an output buffer 4 bytes past a 16-byte boundary (row stride a multiple of 4): scalar stores
    ldy4 = (L + N - 1 + 3) // 4 * 4
    buf = torch.full((C * F * ldy4 + 1,), 7.0, device=DEV)
    y4 = buf[1:].view(C * F, ldy4)
    assert y4.data_ptr() % 16 == 4
    fb.run(torch.from_numpy(x).to(DEV), y=y4, L=L)
    torch.cuda.synchronize()
    assert np.array_equal(y4.view(C, F, ldy4).cpu().numpy()[:, :, :L + N - 1], yc[:, :, :L + N - 1])
    with pytest.raises(apx.ApxError):
        apx.FilterBank(ctx, torch.zeros(33, 10, device=DEV))
    with pytest.raises(apx.ApxError) as e:
        apx.FilterBank(ctx, torch.zeros(4, 513, device=DEV))
    assert e.value.status == apx.APX_E_UNSUPPORTED
    with pytest.raises(apx.ApxError):
        apx.apx_fbank_run(ctx.h, fb.h, torch.from_numpy(x).to(DEV), L, torch.empty(C * F, L, device=DEV))
    fb.close()


@pytest.mark.parametrize("prec", [apx.APX_FB_F16X3, apx.APX_FB_BF16X3])
def test_fbank_full_size(ctx, prec):
    """256 channels of 2^20 pink-noise samples, 32 Hann band-pass filters of 512 taps: sampled
    outputs against FP64 dot products, including the first and last outputs of each row."""
    C, L, F, N = 256, 1 << 20, 32, 512
    x = synth.pink_noise(C, L, 4001)
    h = synth.bandpass_bank(F, N)
    xd = torch.from_numpy(x).to(DEV)
    fb = apx.FilterBank(ctx, torch.from_numpy(h).to(DEV), prec)
    _say(fb.describe())
    Lout = L + N - 1
    y = fb.run(xd, ldy=(Lout + 63) // 64 * 64)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    cs = rng.integers(0, C, 48)
    fs = rng.integers(0, F, 48)
    ts = np.concatenate([rng.integers(0, Lout, 2000), np.arange(0, 600), np.arange(Lout - 600, Lout)])
    K = 512
    coef = 3 * EPS[prec] + (K + 2) * 2.0 ** -24
    num = den = 0.0
    for c, f in zip(cs, fs):
        got = y[c, f, torch.from_numpy(ts).to(DEV)].cpu().numpy().astype(np.float64)
        xs = np.concatenate([np.zeros(N - 1), x[c].astype(np.float64), np.zeros(N - 1)])
        # y[t] = sum_n x[t - n] h[n]: window xs[t .. t + N - 1] against reversed taps
        idx = ts[:, None] + np.arange(N)[None, :]
        win = xs[idx]
        hr = h[f].astype(np.float64)[::-1]
        ref = win @ hr
        bound = coef * (np.abs(win) @ np.abs(hr)) + ABS[prec] * (np.abs(win).sum(axis=1) + np.abs(hr).sum())
        err = np.abs(got - ref)
        num += float(np.sum(ref * ref))
        den += float(np.sum(err * err))
        assert np.all(err <= bound + 1e-30), (c, f, int(np.argmax(err - bound)))
    _say(f"  sampled outputs: SNR vs FP64 {10 * math.log10(num / den):.1f} dB")
    fb.close()
