"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Packed modes: the integer fields r~ are compared bit for bit and the FP32 outputs are compared
bit for bit (both sides multiply the exact integer by (c_s c_k)^-1 in FP64, eq. 16, and round
once to FP32).
Full-precision FP32 paths: within an error bound derived from FP32 arithmetic (gpu_checks.fp32_bound).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1201_3018_amd import synth
from gpu_checks import check_mixed_blocks, fp32_bound as _fp32_bound

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1201_3018_amd import apx  # noqa: E402

DEV = torch.device("cuda:0")
MODES = {O.SYM: apx.APX_SYM, O.ASYM2: apx.APX_ASYM2, O.ASYM3: apx.APX_ASYM3}
CORES = {"td": apx.APX_CORE_TIME, "fft": apx.APX_CORE_FFT, "int8": apx.APX_CORE_INT8}


@pytest.fixture(scope="module")
def ctx():
    c = apx.Context(0)
    yield c
    c.close()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def _say(*a):
    print(*a, flush=True)


def _run_fixed(ctx, s, k, Wb, mode, core, S=0, K=0, op=apx.APX_CONV, variant=apx.FFT_AUTO):
    kern = apx.Kernel(ctx, _dev(k), Wb, mode=MODES.get(mode, mode), core=CORES[core], Sq=S, Kq=K, op=op,
                      fft_variant=variant)
    ts = _dev(s)
    # outputs start as NaN, so that a position no kernel writes cannot pass as a stale value
    out = torch.full((len(s) + len(k) - 1,), float("nan"), dtype=torch.float32, device=DEV)
    out, info = kern.run(ts, out=out, info=True)
    fields = None
    if mode in MODES:
        fields = torch.full((len(s) + len(k) - 1,), float("nan"), dtype=torch.float64, device=DEV)
        apx.apx_debug_fields(ctx.h, kern.h, ts, fields)
    torch.cuda.synchronize()
    res = (out.cpu().numpy(), None if fields is None else fields.cpu().numpy(), apx.block_info(info))
    kern.close()
    return res


def _check_packed(s, k, Wb, mode, S, got, fields, info, kernel_for_oracle=None):
    kk = k if kernel_for_oracle is None else kernel_for_oracle
    ps = O.fixed_params(s, kk, Wb, mode, S, S)
    ref, ref_f, _ = O.conv_blocked(s, kk, Wb, ps, return_fields=True)
    bad = np.nonzero(fields != ref_f)[0]
    assert bad.size == 0, f"{bad.size} integer fields differ, first at {bad[:8]}"
    # bit for bit: a zero digit gives +0 on both sides
    badr = np.nonzero(got.view(np.int32) != ref.view(np.int32))[0]
    assert badr.size == 0, f"{badr.size} outputs differ, first at {badr[:8]}: {got[badr[:4]]} vs {ref[badr[:4]]}"
    # block report
    part = O.partition(len(s), len(k), Wb)
    assert info.size == part.P
    assert np.all(info["Sq"] == S) and np.all(info["Kq"] == S)
    assert np.array_equal(info["cs"], np.array([p.cs for p in ps]))
    assert np.array_equal(info["smax"], np.array([p.smax for p in ps]))
    assert np.allclose(info["rms"], np.array([p.rms for p in ps]), rtol=1e-12, atol=0)


# ------------------------------------------------------------------------- time-domain config
C1 = dict(L=65536, N=64, Wb=1024)


@pytest.mark.parametrize("mode,S", [(O.SYM, 38), (O.ASYM2, 127), (O.ASYM3, 38), (O.ASYM2, 814)])
def test_c1_time_domain_packed(ctx, mode, S):
    _say("case: C1 time domain", mode, "S=K=", S)
    s, k = synth.gaussian(C1["L"], 1001), synth.uniform(C1["N"], 1002)
    got, fields, info = _run_fixed(ctx, s, k, C1["Wb"], mode, "td", S, S)
    _check_packed(s, k, C1["Wb"], mode, S, got, fields, info)
    snr = O.measured_snr_db(got, O.conv_direct(s, k))
    _say(f"  SNR vs FP64 = {snr:.2f} dB")


@pytest.mark.parametrize("core", ["td", "fft"])
def test_c1_full_precision_fp32(ctx, core):
    _say("case: C1 full precision FP32", core)
    s, k = synth.gaussian(C1["L"], 1001), synth.uniform(C1["N"], 1002)
    got, _, info = _run_fixed(ctx, s, k, C1["Wb"], apx.APX_FULL_FP32, core)
    ref = O.conv_direct(s, k)
    err = np.abs(got.astype(np.float64) - ref)
    assert np.all(err <= _fp32_bound(s, k, C1["Wb"], core)), float(np.max(err))
    assert np.all(info["mode"] == apx.APX_FULL_FP32)


def test_c1_full_precision_fp64(ctx):
    _say("case: C1 full precision FP64 time domain")
    s, k = synth.gaussian(C1["L"], 1001), synth.uniform(C1["N"], 1002)
    got, _, _ = _run_fixed(ctx, s, k, C1["Wb"], apx.APX_FULL_FP64, "td")
    ref = O.conv_direct(s, k)
    assert np.array_equal(got, ref.astype(np.float32)) or np.max(np.abs(got - ref.astype(np.float32))) <= \
        2.0 ** -23 * np.max(np.abs(ref))


# ------------------------------------------------------------------------- FFT core, small
VARIANTS = {"block": apx.FFT_BLOCK, "wave": apx.FFT_WAVE, "group": apx.FFT_GROUP}
# shapes whose transform sizes the group core is compiled for (multiples of 512 points)
GROUP_SHAPES = [(4097, 129, 2048), (12000, 300, 2048), (40000, 1024, 4096), (9001, 1000, 4096)]


@pytest.mark.parametrize("variant", ["block", "wave"])
@pytest.mark.parametrize("mode", [O.SYM, O.ASYM2, O.ASYM3])
@pytest.mark.parametrize("L,N,Wb", [(50000, 256, 1024), (9000, 101, 512), (300, 33, 128), (4097, 129, 2048),
                                    (40000, 1024, 4096)])
def test_fft_core_packed_small(ctx, mode, L, N, Wb, variant):
    _say("case: FFT core", variant, mode, L, N, Wb)
    s, k = synth.ar1(L, 11 + N), synth.hann_lowpass(N, 0.2)
    S = O.max_q(mode, N if N % 2 else N + 1)
    got, fields, info = _run_fixed(ctx, s, k, Wb, mode, "fft", S, S, variant=VARIANTS[variant])
    _check_packed(s, k, Wb, mode, S, got, fields, info)


@pytest.mark.parametrize("tail", [2047, 2048, 2049, 3000])
@pytest.mark.parametrize("mode", [O.SYM, O.ASYM2])
def test_wave_window_chunk_edges(ctx, mode, tail):
    """The one-wave core loads its window in chunks of 2048 samples and skips the per-sample
    bounds on a chunk that lies wholly inside the signal.  A last window of 2047..3000 samples
    puts the signal end just before, on and after a chunk edge."""
    N, Wb = 1024, 4096
    W = Wb - (N + 1) - 1
    L = 5 * W - 2 + tail
    part = O.partition(L, N, Wb)
    assert L - int(part.starts[-1]) == tail
    _say("case: wave window chunk edges", mode, L, tail)
    s, k = synth.ar1(L, 700 + tail), synth.hann_lowpass(N)
    S = O.max_q(mode, N + 1)
    got, fields, info = _run_fixed(ctx, s, k, Wb, mode, "fft", S, S, variant=VARIANTS["wave"])
    _check_packed(s, k, Wb, mode, S, got, fields, info)


def test_unaligned_input_rejected(ctx):
    """s_in 4 bytes past an 8-byte boundary (a view one float into a buffer) is rejected on the
    host with APX_E_INVALID before any launch, on every entry point that takes a signal; the
    same data in its own buffer runs."""
    L, N, Wb = 40000, 1024, 4096
    s, k = synth.ar1(L, 93), synth.hann_lowpass(N)
    buf = torch.zeros(L + 1, dtype=torch.float32, device=DEV)
    buf[1:] = _dev(s)
    mis = buf[1:]
    assert mis.data_ptr() % 8 == 4
    S = O.max_q(O.ASYM2, N + 1)
    for core in ("td", "fft", "int8"):
        kern = apx.Kernel(ctx, _dev(k), Wb, mode=apx.APX_ASYM2, core=CORES[core], Sq=S, Kq=S)
        with pytest.raises(apx.ApxError) as e:
            kern.run(mis)
        assert e.value.status == apx.APX_E_INVALID
        kern.run(_dev(s))
        kern.close()
    kauto = apx.Kernel(ctx, _dev(k), Wb, mode=apx.APX_AUTO_SNR, snr_min_db=40.0)
    with pytest.raises(apx.ApxError) as e:
        apx.apx_calibrate(ctx.h, kauto.h, mis, block=1, Q=8)
    assert e.value.status == apx.APX_E_INVALID
    ws = torch.empty(apx.apx_workspace_bytes(), dtype=torch.uint8, device=DEV)
    out = torch.empty(L + N - 1, dtype=torch.float32, device=DEV)
    with pytest.raises(apx.ApxError) as e:
        apx.apx_run_auto(ctx.h, kauto.h, mis, out, 40.0, 1, ws, None)
    assert e.value.status == apx.APX_E_INVALID
    torch.cuda.synchronize()
    kauto.close()


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_wave_nonfinite_in_full_chunk(ctx, bad):
    """A non-finite sample inside a chunk that takes the unguarded loads still flags its
    blocks: their outputs are NaN, every other block equals the oracle."""
    N, Wb, L = 1024, 4096, 30000
    s, k = synth.ar1(L, 731), synth.hann_lowpass(N)
    s[12345] = bad
    _say("case: wave non-finite in a full chunk", bad)
    S = O.max_q(O.ASYM2, N + 1)
    got, _, info = _run_fixed(ctx, s, k, Wb, O.ASYM2, "fft", S, S, variant=VARIANTS["wave"])
    ref = O.conv_blocked(s, k, Wb, O.fixed_params(s, k, Wb, O.ASYM2, S, S))
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    fin = ~np.isnan(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.count_nonzero(info["flags"] & apx.APX_FLAG_NONFINITE) >= 1


@pytest.mark.parametrize("mode,N,Wb", [(O.ASYM2, 800, 8994), (O.ASYM3, 800, 8994), (O.SYM, 800, 8994),
                                       (O.SYM, 800, 17186),
                                       (O.ASYM2, 800, 17186), (O.ASYM3, 800, 17186), (O.ASYM3, 800, 33570),
                                       (O.SYM, 101, 32768), (O.ASYM2, 40, 600)])
def test_fft_block_core_own_length(ctx, mode, N, Wb):
    """LDS core of one fixed packed mode at the transform length of its own words (W_block / 2
    symmetric, T + N - 1 asymmetric), up to the longest transform one workgroup holds (16384
    words, W_block beyond 16384): three blocks and a ragged tail, U[-128, 128] inputs."""
    No = N if N % 2 else N + 1
    L = 3 * (Wb - No - 1) + 555
    _say("case: FFT block core, own length", mode, L, N, Wb)
    s = synth.uniform(L, 51 + N) * np.float32(128.0)
    k = synth.uniform(N, 52 + N) * np.float32(128.0)
    S = O.max_q(mode, No)
    kern = apx.Kernel(ctx, _dev(k), Wb, mode=MODES[mode], core=apx.APX_CORE_FFT, Sq=S, Kq=S,
                      fft_variant=apx.FFT_BLOCK)
    desc = kern.describe()
    kern.close()
    _say(" ", desc)
    assert "k_fft1" in desc
    got, fields, info = _run_fixed(ctx, s, k, Wb, mode, "fft", S, S, variant=apx.FFT_BLOCK)
    _check_packed(s, k, Wb, mode, S, got, fields, info)


def test_fft_block_core_limits(ctx):
    """Beyond one workgroup's transform (16384 words) the multi-pass core takes over (FP32 above
    W_block = 16384, symmetric above 32768, asymmetric M=2 above 16384 words), up to 65536 words
    (131072 for FP32); beyond that the FFT core refuses."""
    k = _dev(synth.uniform(800, 9))
    for mode, Wb in ((apx.APX_FULL_FP32, 17186), (apx.APX_ASYM2, 33570), (apx.APX_SYM, 33570)):
        kern = apx.Kernel(ctx, k, Wb, mode=mode, core=apx.APX_CORE_FFT)
        assert "k_big" in kern.describe(), (mode, Wb, kern.describe())
        kern.close()
    for mode, Wb in ((apx.APX_FULL_FP32, 131074), (apx.APX_ASYM2, 131072), (apx.APX_SYM, 131074)):
        with pytest.raises(apx.ApxError) as e:
            apx.Kernel(ctx, k, Wb, mode=mode, core=apx.APX_CORE_FFT)
        assert e.value.status == apx.APX_E_UNSUPPORTED, (mode, Wb)


@pytest.mark.parametrize("mode", [O.SYM, O.ASYM2, O.ASYM3])
@pytest.mark.parametrize("L,N,Wb", GROUP_SHAPES)
def test_fft_group_packed(ctx, mode, L, N, Wb):
    _say("case: FFT core, group", mode, L, N, Wb)
    s, k = synth.ar1(L, 31 + N), synth.hann_lowpass(N, 0.2)
    S = O.max_q(mode, N if N % 2 else N + 1)
    got, fields, info = _run_fixed(ctx, s, k, Wb, mode, "fft", S, S, variant=apx.FFT_GROUP)
    _check_packed(s, k, Wb, mode, S, got, fields, info)


def test_fft_group_fp32_and_edges(ctx):
    for L, N, Wb in GROUP_SHAPES:
        _say("case: FP32 group", L, N, Wb)
        s, k = synth.ar1(L, 6), synth.hann_lowpass(N, 0.1)
        got, _, _ = _run_fixed(ctx, s, k, Wb, apx.APX_FULL_FP32, "fft", variant=apx.FFT_GROUP)
        err = np.abs(got.astype(np.float64) - O.conv_direct(s, k))
        assert np.all(err <= _fp32_bound(s, k, Wb, "fft")), (L, N, Wb, float(np.max(err)))
    _say("case: zero / non-finite blocks, group")
    s = synth.gaussian(30000, 7)
    s[5000:9000] = 0.0
    s[20000] = np.inf
    k = synth.uniform(129, 8)
    got, fields, info = _run_fixed(ctx, s, k, 2048, O.ASYM2, "fft", variant=apx.FFT_GROUP)
    S = O.max_q(O.ASYM2, 129)
    ref = O.conv_blocked(s, k, 2048, O.fixed_params(s, k, 2048, O.ASYM2, S, S))
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    fin = ~np.isnan(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.any(info["flags"] & apx.APX_FLAG_NONFINITE) and np.any(info["flags"] & apx.APX_FLAG_ZERO)
    with pytest.raises(apx.ApxError) as e:
        _run_fixed(ctx, s, k[:31], 256, O.SYM, "fft", variant=apx.FFT_GROUP)
    assert e.value.status == apx.APX_E_UNSUPPORTED


@pytest.mark.parametrize("mode", [O.SYM, O.ASYM2, O.ASYM3])
@pytest.mark.parametrize("L,N,Wb", [(20000, 64, 1024), (9000, 101, 512), (1, 1, 8), (7, 7, 64), (40, 40, 256)])
def test_td_core_packed_small(ctx, mode, L, N, Wb):
    _say("case: TD core", mode, L, N, Wb)
    s, k = synth.gaussian(L, 21 + N), synth.uniform(N, 22 + N)
    S = O.max_q(mode, N if N % 2 else N + 1)
    got, fields, info = _run_fixed(ctx, s, k, Wb, mode, "td", S, S)
    _check_packed(s, k, Wb, mode, S, got, fields, info)


@pytest.mark.parametrize("mode", [O.SYM, O.ASYM2])
@pytest.mark.parametrize("N", [128, 257, 512, 1024])
def test_td_core_long_kernels(ctx, mode, N):
    """Time-domain core at the kernel lengths of the time-domain sweep (W_block = max(2N, 1024)
    + N + 1), several blocks and a ragged tail."""
    No = N if N % 2 else N + 1
    Wb = max(2 * No, 1024) + No + 1
    L = 3 * (Wb - No - 1) + 777
    _say("case: TD long kernel", mode, L, N, Wb)
    s, k = synth.gaussian(L, 41 + N), synth.uniform(N, 42 + N)
    S = O.max_q(mode, No)
    got, fields, info = _run_fixed(ctx, s, k, Wb, mode, "td", S, S)
    _check_packed(s, k, Wb, mode, S, got, fields, info)


@pytest.mark.parametrize("core,variant", [("td", "block"), ("fft", "block"), ("fft", "wave")])
def test_fp32_small_shapes(ctx, core, variant):
    for L, N, Wb in [(9000, 101, 512), (300, 33, 128), (4097, 129, 2048), (1000, 64, 1024), (40000, 1024, 4096)]:
        _say("case: FP32", core, variant, L, N, Wb)
        s, k = synth.ar1(L, 5), synth.hann_lowpass(N, 0.1)
        got, _, _ = _run_fixed(ctx, s, k, Wb, apx.APX_FULL_FP32, core, variant=VARIANTS[variant])
        ref = O.conv_direct(s, k)
        err = np.abs(got.astype(np.float64) - ref)
        assert np.all(err <= _fp32_bound(s, k, Wb, core)), (L, N, Wb, float(np.max(err)))


# ------------------------------------------------------------------------- edge cases
@pytest.mark.parametrize("core,variant", [("td", "block"), ("fft", "block"), ("fft", "wave"), ("int8", "block")])
def test_zero_and_nonfinite_blocks(ctx, core, variant):
    _say("case: zero / non-finite blocks", core, variant)
    s = synth.gaussian(10000, 3)
    s[1000:3000] = 0.0
    s[7000] = np.nan
    k = synth.uniform(31, 4)
    got, fields, info = _run_fixed(ctx, s, k, 256, O.SYM, core, 20, 20, variant=VARIANTS[variant])
    ref = O.conv_blocked(s, k, 256, O.fixed_params(s, k, 256, O.SYM, 20, 20))
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    fin = ~np.isnan(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.any(info["flags"] & apx.APX_FLAG_NONFINITE)
    assert np.any(info["flags"] & apx.APX_FLAG_ZERO)


@pytest.mark.parametrize("core", ["td", "fft"])
def test_xcorr_matches_reversed_conv_and_textbook(ctx, core):
    _say("case: correlation", core)
    s, k = synth.ar1(6000, 8), synth.gaussian(65, 9)
    S = O.max_q(O.SYM, 65)
    got, fields, info = _run_fixed(ctx, s, k, 512, O.SYM, core, S, S, op=apx.APX_XCORR)
    _check_packed(s, k, 512, O.SYM, S, got, fields, info, kernel_for_oracle=k[::-1].copy())
    # against the textbook correlation in full precision (quantization error only)
    ref = O.xcorr(s, k)
    assert O.measured_snr_db(got, ref) > 25.0
    g32, _, _ = _run_fixed(ctx, s, k, 512, apx.APX_FULL_FP32, core, op=apx.APX_XCORR)
    assert np.max(np.abs(g32 - ref)) < 1e-4 * np.max(np.abs(ref))
    assert np.argmax(g32) == np.argmax(ref)


def test_errors_reported(ctx):
    k = _dev(synth.uniform(64, 1))
    with pytest.raises(apx.ApxError) as e:
        apx.Kernel(ctx, k, 1024, mode=apx.APX_SYM, Sq=127, Kq=127)      # 65*127^2 > 97667
    assert e.value.status == apx.APX_E_BOUND
    with pytest.raises(apx.ApxError) as e:
        apx.Kernel(ctx, k, 1025, mode=apx.APX_SYM)                     # W odd
    assert e.value.status == apx.APX_E_INVALID
    big = 2 ** 31 - 1                                                  # N S K wraps past 2^63
    for unsafe in (False, True):
        with pytest.raises(apx.ApxError) as e:
            apx.Kernel(ctx, _dev(synth.uniform(3, 2)), 32, mode=apx.APX_SYM, Sq=big, Kq=big, allow_unsafe=unsafe)
        assert e.value.status == apx.APX_E_BOUND, unsafe
    kern = apx.Kernel(ctx, k, 1024, mode=apx.APX_SYM)
    with pytest.raises(apx.ApxError):
        kern.run(_dev(np.zeros(10, np.float32)))                       # L < N
    kern.close()
    # the bound is there for a reason: forced beyond it, unpacking goes wrong
    s = synth.gaussian(8192, 1001)
    kern = apx.Kernel(ctx, k, 1024, mode=apx.APX_SYM, Sq=127, Kq=127, allow_unsafe=True, core=apx.APX_CORE_TIME)
    f = kern.fields(_dev(s)).cpu().numpy()
    kern.close()
    assert np.sum(f != O.int_fields(s, synth.uniform(64, 1), 1024, 127, 127)) > 100


# ------------------------------------------------------------------------- full-size FFT config
@pytest.fixture(scope="module")
def c2():
    s = synth.ar1(1 << 22, 2001)
    k = synth.hann_lowpass(1024)
    return s, k


@pytest.mark.parametrize("variant", ["block", "wave", "group"])
@pytest.mark.parametrize("mode,S", [(O.ASYM2, 205), (O.SYM, 9), (O.ASYM3, 9)])
def test_c2_fft_full_size(ctx, c2, mode, S, variant):
    _say("case: C2 full size FFT", variant, mode, S)
    s, k = c2
    got, fields, info = _run_fixed(ctx, s, k, 4096, mode, "fft", S, S, variant=VARIANTS[variant])
    _check_packed(s, k, 4096, mode, S, got, fields, info)


@pytest.mark.parametrize("mode,S", [(O.ASYM2, 205), (O.SYM, 9), (O.ASYM3, 9), (O.ASYM2, 127), (O.SYM, 16)])
def test_c2_int8_full_size(ctx, c2, mode, S):
    """Integer matrix-core core on the FFT-block workload: every output and every integer field
    equal to the oracle's, including symmetric S_q = K_q = 16 beyond Table 1's bound (no packing
    here), and equal to the packed FFT core where that one is exact."""
    _say("case: C2 full size int8 core", mode, S)
    s, k = c2
    got, fields, info = _run_fixed(ctx, s, k, 4096, mode, "int8", S, S)
    _check_packed(s, k, 4096, mode, S, got, fields, info)
    if O.max_q(mode, 1025) >= S:
        fft, _, _ = _run_fixed(ctx, s, k, 4096, mode, "fft", S, S)
        assert np.array_equal(got, fft)  # equal values (a zero may carry either sign)


@pytest.mark.parametrize("mode,S", [(O.SYM, 0), (O.ASYM2, 0), (O.ASYM3, 0), (O.ASYM2, 127), (O.SYM, 40),
                                    (O.ASYM2, 300), (O.ASYM3, 16319)])
@pytest.mark.parametrize("L,N,Wb", [(50000, 256, 1024), (9000, 101, 512), (300, 33, 128), (7, 7, 64),
                                    (40000, 1024, 4096), (30001, 2000, 8192), (5000, 64, 20000)])
def test_int8_core_small(ctx, mode, S, L, N, Wb):
    """Integer core against the oracle: several tiles per block, ragged tails, block 0's leading
    outputs, one-digit and two-digit operands (S_q above 127), S_q beyond the packing bounds."""
    No = N if N % 2 else N + 1
    Sq = S or O.max_q(mode, No)
    _say("case: int8 core", mode, Sq, L, N, Wb)
    s, k = synth.ar1(L, 61 + N), synth.hann_lowpass(N, 0.2)
    got, fields, info = _run_fixed(ctx, s, k, Wb, mode, "int8", Sq, Sq)
    _check_packed(s, k, Wb, mode, Sq, got, fields, info)


def test_int8_core_xcorr_and_errors(ctx):
    s, k = synth.gaussian(30000, 71), synth.uniform(300, 72)
    S = O.max_q(O.ASYM2, 301)
    got, fields, info = _run_fixed(ctx, s, k, 2048, O.ASYM2, "int8", S, S, op=apx.APX_XCORR)
    _check_packed(s, k, 2048, O.ASYM2, S, got, fields, info, kernel_for_oracle=k[::-1].copy())
    tk = _dev(k)
    for mode, kw in ((apx.APX_FULL_FP32, {}), (apx.APX_AUTO_SNR, {"snr_min_db": 30.0}),
                     (apx.APX_ASYM2, {"Sq": 16320, "Kq": 16320})):
        with pytest.raises(apx.ApxError) as e:
            apx.Kernel(ctx, tk, 2048, mode=mode, core=apx.APX_CORE_INT8, **kw)
        assert e.value.status == apx.APX_E_UNSUPPORTED, mode


@pytest.mark.parametrize("target", [40.0, 50.0])
def test_c2_auto_snr_selection(ctx, c2, target):
    """Per-block choice on the FFT-block workload: modes equal the oracle's selection except at
    exact ties of the model SNR with the target; packed blocks equal the oracle bit for bit and
    FP32 blocks lie within the FP32 bound.  At 50 dB every block runs FP32 inside the per-block
    choice kernel."""
    _say(f"case: C2 SNR-driven selection at {target} dB")
    s, k = c2
    ts, tk = _dev(s), _dev(k)
    calib_o = O.calibrate(s, k, 4096)
    kern = apx.Kernel(ctx, tk, 4096, mode=apx.APX_AUTO_SNR, core=apx.APX_CORE_FFT, snr_min_db=target)
    calib_g = kern.calibrate(ts)
    assert abs(calib_g - calib_o) < 1e-6
    out, info = kern.run(ts, info=True)
    torch.cuda.synchronize()
    got, info = out.cpu().numpy(), apx.block_info(info)
    kern.close()
    ps = O.auto_params(s, k, 4096, target, calib_g)
    want = np.array([{O.SYM: 1, O.ASYM2: 2, O.FULL: 0}[p.mode] for p in ps])
    near = np.array([abs(p.snr_pred_db - target) < 1e-6 for p in ps])
    assert np.array_equal(info["mode"][~near], want[~near])
    ref64 = O.conv_direct(s, k)
    n_packed, n_fp32 = check_mixed_blocks(s, k, 4096, ps, info["mode"], got, "fft", ref64)
    part = O.partition(len(s), len(k), 4096)
    snrs = []
    for w in range(part.P):
        j_lo, j_hi, o = part.keep(w)
        sl = slice(o, o + j_hi - j_lo)
        snrs.append(O.measured_snr_db(got[sl], ref64[sl]))
    snrs = np.array(snrs)
    _say(f"  modes: {np.bincount(info['mode'], minlength=3)} ({n_packed} packed, {n_fp32} FP32); "
         f"measured SNR min {snrs.min():.2f} mean {snrs.mean():.2f}")
    assert np.all(snrs[info["mode"] != 0] >= target - 3.0)
    if target == 50.0:
        assert n_fp32 == part.P


# ------------------------------------------------------------------------- tie of a base digit
def _tie_case(L=20000, N=65, Wb=1024, seed=77):
    """A signal with full-scale alternating segments of N samples against the alternating kernel
    k[n] = (-1)^n: the output at the segment's last sample is +-N S K = +-R_max, the only value
    of a symmetric word's base digit at which two digit splits give the same word (the
    no-overlap condition excludes it).  Every other output stays below R_max, because the rest of
    the signal stays below 0.9 of full scale.  Returns s, k and the tie positions (odd: a base
    digit; even: a plain output at R_max, not a tie)."""
    rng = np.random.default_rng(seed)
    s = rng.uniform(-0.9, 0.9, L).astype(np.float32)
    k = np.where(np.arange(N) % 2 == 0, 1.0, -1.0).astype(np.float32)
    part = O.partition(L, N, Wb)
    ends = []
    for t, m in enumerate([N - 1 + 2 * 101 + 1, 3 * part.W + 40 + 1, 5 * part.W + 500, 8 * part.W + 7 + 1,
                           11 * part.W + N - 1 + 1, L - 3]):
        a = m - (N - 1)
        sign = 1.0 if t % 2 == 0 else -1.0
        s[a: m + 1] = sign * np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
        ends.append(m)
    return s, k, ends


@pytest.mark.parametrize("core,variant", [("td", apx.FFT_AUTO), ("fft", apx.FFT_BLOCK), ("fft", apx.FFT_WAVE),
                                          ("fft", apx.FFT_GROUP), ("int8", apx.FFT_AUTO)])
def test_sym_base_digit_tie(ctx, core, variant):
    """Symmetric packing with a base digit at +-R_max.  The word 2R D + B + eps E holds the same
    value for (D, R) and (D + 1, -R), so the unpacking cannot tell which one the convolution
    produced.  Every output other than the tied digit and the output of its word's upper digit
    equals the plain definition; those two are either exact or the other split (D + d, B - 2R d),
    d = +-1, with the same word value.  The integer core does not pack and is exact everywhere;
    even positions at R_max are no tie and are exact on every core.  The FFT cores run at
    S_q = K_q = 16: the coherent full-scale segments make their rounding error large, and at the
    largest in-bound S_q = K_q (38) it moves side digits of outputs near the segments (Table 1's
    bound is the one for the sequential time-domain sum); the ties are there at any S_q."""
    N, Wb = 65, (2048 if variant == apx.FFT_GROUP else 1024)  # the group core's smallest block
    s, k, ends = _tie_case(L=20000 * Wb // 1024, N=N, Wb=Wb)
    S = 16 if core == "fft" else O.max_q(O.SYM, N)
    _say("case: symmetric base-digit tie", core, variant, "S=K=", S, "ends", ends)
    got, fields, info = _run_fixed(ctx, s, k, Wb, O.SYM, core, S, S, variant=variant)
    ps = O.fixed_params(s, k, Wb, O.SYM, S, S)
    ref, ref_f, cks = O.conv_blocked(s, k, Wb, ps, return_fields=True)
    R = O.r_max(N, S, S)
    assert [abs(int(ref_f[m])) for m in ends] == [R] * len(ends)
    assert int(np.count_nonzero(np.abs(ref_f) == R)) == len(ends)
    loose = set()
    for m in ends:
        if m % 2 == 1 and core != "int8":
            loose.update((m - 1, m))
    mask = np.ones(ref.size, bool)
    mask[sorted(loose)] = False
    bad = np.nonzero(fields[mask] != ref_f[mask])[0]
    assert bad.size == 0, f"{bad.size} fields differ away from the ties, first at {np.nonzero(mask)[0][bad[:4]]}"
    assert np.array_equal(got[mask], ref[mask])
    part = O.partition(len(s), N, Wb)
    ck = cks[S]
    n_split = 0
    for m in ends:
        if (m - 1) not in loose:
            continue
        w = next(w for w in range(part.P) if part.keep(w)[2] <= m < part.keep(w)[2] + part.keep(w)[1] - part.keep(w)[0])
        inv = 1.0 / (ps[w].cs * ck)
        if fields[m] == ref_f[m] and fields[m - 1] == ref_f[m - 1]:
            assert got[m] == ref[m] and got[m - 1] == ref[m - 1]
            continue
        d = int(fields[m - 1] - ref_f[m - 1])
        assert d in (-1, 1) and fields[m] == ref_f[m] - 2 * R * d, (m, fields[m - 1:m + 1], ref_f[m - 1:m + 1])
        assert got[m - 1] == np.float32(inv * float(fields[m - 1])) and got[m] == np.float32(inv * float(fields[m]))
        n_split += 1
    _say(f"  {n_split} of {len(loose) // 2} base-digit ties took the other split")
