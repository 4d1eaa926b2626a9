"""Parity of the multi-pass FFT core (transforms through a device scratch, for blocks beyond one
workgroup's LDS) against the oracle, through the C ABI.

Packed modes: integer fields and outputs bit for bit against the plain per-block definition.
FP32: within the FP32 bound of gpu_checks.fp32_bound.  Forced (fft_variant 4) at small sizes with a
ragged tail and block 0's prefix item, and taken by itself at W_block = 32768 and 65536 (the
largest block sizes of the paper's sweep, Section IV.A).
"""
import numpy as np
import pytest

import oracle as O
from paper_1201_3018_amd import synth
from gpu_checks import fp32_bound

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


def _run(ctx, s, k, Wb, mode, S=0, variant=apx.FFT_AUTO):
    kern = apx.Kernel(ctx, _dev(k), Wb, mode=MODES.get(mode, mode), core=apx.APX_CORE_FFT, Sq=S, Kq=S,
                      fft_variant=variant)
    desc = kern.describe()
    ts = _dev(s)
    out = torch.full((len(s) + len(k) - 1,), float("nan"), dtype=torch.float32, device=DEV)
    out, info = kern.run(ts, out=out, info=True)
    fields = None
    if mode in MODES:
        fields = torch.full((len(s) + len(k) - 1,), float("nan"), dtype=torch.float64, device=DEV)
        apx.apx_debug_fields(ctx.h, kern.h, ts, fields)
    torch.cuda.synchronize()
    res = (out.cpu().numpy(), None if fields is None else fields.cpu().numpy(), apx.block_info(info), desc)
    kern.close()
    return res


def _check_packed(s, k, Wb, mode, S, got, fields, info):
    ps = O.fixed_params(s, k, Wb, mode, S, S)
    ref, ref_f, _ = O.conv_blocked(s, k, Wb, ps, return_fields=True)
    bad = np.nonzero(fields != ref_f)[0]
    assert bad.size == 0, f"{bad.size} integer fields differ, first at {bad[:8]}"
    badr = np.nonzero(got.view(np.int32) != ref.view(np.int32))[0]
    assert badr.size == 0, f"{badr.size} outputs differ, first at {badr[:8]}"
    assert info.size == O.partition(len(s), len(k), Wb).P
    assert np.array_equal(info["cs"], np.array([p.cs for p in ps]))


# transforms of 2^10 to 2^13 points (the smallest the core takes: 2048 words)
SMALL = [(30001, 129, 4096), (70000, 1001, 8192), (90001, 300, 16384)]


@pytest.mark.parametrize("mode", [O.SYM, O.ASYM2, O.ASYM3])
@pytest.mark.parametrize("L,N,Wb", SMALL)
def test_multipass_forced_packed(ctx, mode, L, N, Wb):
    s, k = synth.ar1(L, 41 + N), synth.hann_lowpass(N, 0.2)
    S = O.max_q(mode, N if N % 2 else N + 1)
    got, fields, info, desc = _run(ctx, s, k, Wb, mode, S, variant=apx.FFT_MULTIPASS)
    _say("case: multi-pass forced", mode, L, N, Wb, desc)
    assert "k_big" in desc
    _check_packed(s, k, Wb, mode, S, got, fields, info)


@pytest.mark.parametrize("L,N,Wb", SMALL)
def test_multipass_forced_fp32(ctx, L, N, Wb):
    s, k = synth.ar1(L, 7 + N), synth.hann_lowpass(N, 0.1)
    got, _, _, desc = _run(ctx, s, k, Wb, apx.APX_FULL_FP32, variant=apx.FFT_MULTIPASS)
    _say("case: multi-pass forced FP32", L, N, Wb, desc)
    err = np.abs(got.astype(np.float64) - O.conv_direct(s, k))
    assert np.all(err <= fp32_bound(s, k, Wb, "fft")), float(np.nanmax(err))


@pytest.mark.parametrize("Wb", [32768, 65536])
@pytest.mark.parametrize("mode", [O.SYM, O.ASYM2, O.ASYM3])
def test_multipass_large_blocks_packed(ctx, mode, Wb):
    """The paper's largest block sizes at N = 801, uniform samples (Section IV.A), the largest
    in-bound S_q = K_q; a few blocks and a ragged tail."""
    L, N = 3 * Wb + 12345, 801
    rng = np.random.default_rng(Wb + len(mode))
    s = rng.uniform(-128.0, 128.0, L).astype(np.float32)
    k = rng.uniform(-128.0, 128.0, N).astype(np.float32)
    S = O.max_q(mode, N)
    got, fields, info, desc = _run(ctx, s, k, Wb, mode, S)
    _say("case: multi-pass", mode, "W_block", Wb, desc)
    W = Wb - N - 1
    words = Wb // 2 if mode == O.SYM else -(-W // (2 if mode == O.ASYM2 else 3)) + N - 1
    assert ("k_big" in desc) == (words > 16384), desc  # beyond the one-workgroup transforms only
    _check_packed(s, k, Wb, mode, S, got, fields, info)


@pytest.mark.parametrize("Wb", [32768, 65536, 66338])
def test_multipass_large_blocks_fp32(ctx, Wb):
    L, N = 3 * Wb + 999, 801
    rng = np.random.default_rng(Wb)
    s = rng.uniform(-128.0, 128.0, L).astype(np.float32)
    k = rng.uniform(-128.0, 128.0, N).astype(np.float32)
    got, _, _, desc = _run(ctx, s, k, Wb, apx.APX_FULL_FP32)
    _say("case: multi-pass FP32 W_block", Wb, desc)
    assert "k_big" in desc
    err = np.abs(got.astype(np.float64) - O.conv_direct(s, k))
    assert np.all(err <= fp32_bound(s, k, Wb, "fft")), float(np.nanmax(err))


def test_multipass_zero_nonfinite_and_errors(ctx):
    s = synth.gaussian(40000, 3)
    s[8000:20000] = 0.0
    s[30000] = np.nan
    k = synth.uniform(257, 4)
    S = O.max_q(O.ASYM2, 257)
    got, fields, info, _ = _run(ctx, s, k, 4096, O.ASYM2, S, variant=apx.FFT_MULTIPASS)
    ref = O.conv_blocked(s, k, 4096, O.fixed_params(s, k, 4096, O.ASYM2, S, S))
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    fin = ~np.isnan(ref)
    assert np.array_equal(got[fin].view(np.int32), ref[fin].view(np.int32))
    assert np.any(info["flags"] & apx.APX_FLAG_NONFINITE) and np.any(info["flags"] & apx.APX_FLAG_ZERO)
    # per-block choice is not a multi-pass mode; nor are many signals in one launch
    with pytest.raises(apx.ApxError) as e:
        apx.Kernel(ctx, _dev(k), 4096, mode=apx.APX_AUTO_SNR, core=apx.APX_CORE_FFT, snr_min_db=40.0,
                   fft_variant=apx.FFT_MULTIPASS)
    assert e.value.status == apx.APX_E_UNSUPPORTED
    kern = apx.Kernel(ctx, _dev(k), 4096, mode=apx.APX_ASYM2, core=apx.APX_CORE_FFT, fft_variant=apx.FFT_MULTIPASS)
    with pytest.raises(apx.ApxError) as e:
        apx.Many(kern, [_dev(s), _dev(s)])
    assert e.value.status == apx.APX_E_UNSUPPORTED
    kern.close()
