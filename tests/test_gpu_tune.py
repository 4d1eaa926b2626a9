"""Autotuner (apx_tune): every core / FFT implementation that can run a shape is timed, the
fastest is recorded in the context's table and the table file, kernels created afterwards with
automatic choices use it (W_block = 0 takes the tuned block size), a second process loads the
table, and the tuned kernel's outputs equal the oracle's."""
import os
import subprocess
import sys

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
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def test_tune_choose_block_and_core(tmp_path, monkeypatch):
    path = str(tmp_path / "tune.txt")
    monkeypatch.setenv("APX_TUNE_FILE", path)
    ctx = apx.Context(0)
    N = 64
    k = synth.uniform(N, 1002)
    tk = _dev(k)
    res = apx.apx_tune(ctx.h, tk, 0, apx.params(apx.APX_ASYM2))
    print("tuned:", res, flush=True)
    print(apx.apx_tune_describe(ctx.h), flush=True)
    assert res["W_block"] in (256, 512, 1024) and res["core"] in (apx.APX_CORE_TIME, apx.APX_CORE_INT8, apx.APX_CORE_FFT)
    assert os.path.exists(path)
    kern = apx.Kernel(ctx, tk, 0, mode=apx.APX_ASYM2)
    assert kern.W_block == res["W_block"]
    core_name = {apx.APX_CORE_TIME: "core=time", apx.APX_CORE_INT8: "core=int8", apx.APX_CORE_FFT: "core=fft"}
    assert kern.describe().startswith(core_name[res["core"]]), kern.describe()
    if res["core"] == apx.APX_CORE_INT8:  # the tuned count of output tiles per pass is used
        assert res["tile"] in (1, 2, 3) and f"tiles_per_pass={res['tile']}" in kern.describe(), kern.describe()
    elif res["core"] == apx.APX_CORE_TIME:  # and the tuned outputs per thread
        assert res["tile"] in (4, 8) and f"outputs_per_thread={res['tile']}" in kern.describe(), kern.describe()
    else:
        assert res["tile"] == 0
    s = synth.gaussian(50000, 1001)
    out = torch.full((s.size + N - 1,), float("nan"), dtype=torch.float32, device=DEV)
    kern.run(_dev(s), out=out)
    got = out.cpu().numpy()
    S = O.max_q(O.ASYM2, N + 1)
    ref = O.conv_blocked(s, k, kern.W_block, O.fixed_params(s, k, kern.W_block, O.ASYM2, S, S))
    assert np.array_equal(got.view(np.int32), ref.view(np.int32))
    kern.close()
    # the FFT-block shape: the tuner picks among the FFT core's implementations
    k2 = _dev(synth.hann_lowpass(1024))
    res2 = apx.apx_tune(ctx.h, k2, 4096, apx.params(apx.APX_AUTO_SNR, snr_min_db=40.0), L_hint=1 << 22)
    print("tuned C2 shape:", res2, flush=True)
    assert res2["core"] == apx.APX_CORE_FFT and res2["W_block"] == 4096
    kern2 = apx.Kernel(ctx, k2, 4096, mode=apx.APX_AUTO_SNR, snr_min_db=40.0)
    want = {1: ("k_fft<", "k_fft1<"), 2: ("k_fftw<",), 3: ("k_fftg<",)}[res2["fft_variant"]]
    assert any(w in kern2.describe() for w in want), kern2.describe()
    kern2.close()
    ctx.close()
    # a second process starts with the table
    code = ("import sys; sys.path.insert(0, %r); from paper_1201_3018_amd import apx; c = apx.Context(0); "
            "print(apx.apx_tune_describe(c.h)); c.close()" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                         env=dict(os.environ, APX_TUNE_FILE=path))
    print(out.stdout, flush=True)
    assert out.returncode == 0, out.stderr
    assert f"N=65 op=0 mode={apx.APX_ASYM2} W_block=0" in out.stdout
    assert "N=1025 op=0 mode=4 W_block=4096" in out.stdout


@pytest.mark.parametrize("mode,S", [(O.SYM, 0), (O.ASYM2, 300), (O.ASYM3, 0)])
@pytest.mark.parametrize("L,N,Wb", [(50000, 256, 4096), (20001, 65, 1024)])
def test_int8_tiles_per_pass_from_table(tmp_path, monkeypatch, mode, S, L, N, Wb):
    """The integer core with one, two and three output tiles per pass over the taps, each taken
    from a table entry (the way a tuned choice reaches a kernel), equal to the oracle bit for bit:
    blocks of four tiles (passes of 1, 2 and 3 + 1 tiles) and of one tile, one-digit and two-digit
    operands."""
    No = N if N % 2 else N + 1
    Sq = S or O.max_q(mode, No)
    ctx = apx.Context(0)
    arch = apx.apx_tune_describe(ctx.h).split(",")[0].split()[1]
    ctx.close()
    s, k = synth.ar1(L, 17 + N), synth.hann_lowpass(N, 0.3)
    ref = O.conv_blocked(s, k, Wb, O.fixed_params(s, k, Wb, mode, Sq, Sq))
    amode = {O.SYM: apx.APX_SYM, O.ASYM2: apx.APX_ASYM2, O.ASYM3: apx.APX_ASYM3}[mode]
    for tile in (1, 2, 3):
        path = str(tmp_path / f"tune{tile}.txt")
        with open(path, "w") as f:
            f.write(f"{arch} {No} {apx.APX_CONV} {amode} {Wb} {apx.APX_CORE_INT8} 0 {Wb} 1.000 {tile}\n")
        monkeypatch.setenv("APX_TUNE_FILE", path)
        ctx = apx.Context(0)
        kern = apx.Kernel(ctx, _dev(k), Wb, mode=amode, Sq=Sq, Kq=Sq)
        desc = kern.describe()
        print("case: int8 tiles per pass", tile, mode, Sq, L, N, Wb, desc, flush=True)
        assert desc.startswith("core=int8") and f"tiles_per_pass={tile}" in desc, desc
        out = torch.full((L + N - 1,), float("nan"), dtype=torch.float32, device=DEV)
        kern.run(_dev(s), out=out)
        got = out.cpu().numpy()
        bad = np.nonzero(got.view(np.int32) != ref.view(np.int32))[0]
        assert bad.size == 0, f"tiles {tile}: {bad.size} outputs differ, first at {bad[:8]}"
        kern.close()
        ctx.close()


@pytest.mark.parametrize("mode,S", [(O.SYM, 0), (O.ASYM2, 0), (O.ASYM3, 0), (O.FULL, 0)])
@pytest.mark.parametrize("L,N,Wb", [(50000, 256, 1024), (30001, 33, 4096), (20001, 65, 2048)])
def test_td_outputs_per_thread_from_table(tmp_path, monkeypatch, mode, S, L, N, Wb):
    """The time-domain core with 4 and with 8 outputs per thread, each taken from a table entry:
    packed modes equal the oracle bit for bit, FP32 lies within the FP32 bound of the FP64 sum
    (the FMA order per output is the same for both tiles, so their FP32 outputs are equal too)."""
    from gpu_checks import fp32_bound
    No = N if N % 2 else N + 1
    ctx = apx.Context(0)
    arch = apx.apx_tune_describe(ctx.h).split(",")[0].split()[1]
    ctx.close()
    s, k = synth.ar1(L, 23 + N), synth.hann_lowpass(N, 0.25)
    amode = {O.SYM: apx.APX_SYM, O.ASYM2: apx.APX_ASYM2, O.ASYM3: apx.APX_ASYM3, O.FULL: apx.APX_FULL_FP32}[mode]
    Sq = S or (O.max_q(mode, No) if mode != O.FULL else 0)
    if mode != O.FULL:
        ref = O.conv_blocked(s, k, Wb, O.fixed_params(s, k, Wb, mode, Sq, Sq))
    else:
        ref64, bound = O.conv_direct(s, k), fp32_bound(s, k, Wb, "td")
    outs = []
    for tile in (4, 8):
        path = str(tmp_path / f"tune{tile}.txt")
        with open(path, "w") as f:
            f.write(f"{arch} {No} {apx.APX_CONV} {amode} {Wb} {apx.APX_CORE_TIME} 0 {Wb} 1.000 {tile}\n")
        monkeypatch.setenv("APX_TUNE_FILE", path)
        ctx = apx.Context(0)
        kern = apx.Kernel(ctx, _dev(k), Wb, mode=amode, Sq=Sq, Kq=Sq)
        desc = kern.describe()
        print("case: time-domain outputs per thread", tile, mode, Sq, L, N, Wb, desc, flush=True)
        assert desc.startswith("core=time") and f"outputs_per_thread={tile}" in desc, desc
        out = torch.full((L + N - 1,), float("nan"), dtype=torch.float32, device=DEV)
        kern.run(_dev(s), out=out)
        got = out.cpu().numpy()
        if mode != O.FULL:
            bad = np.nonzero(got.view(np.int32) != ref.view(np.int32))[0]
            assert bad.size == 0, f"tile {tile}: {bad.size} outputs differ, first at {bad[:8]}"
        else:
            err = np.abs(got.astype(np.float64) - ref64)
            assert np.all(err <= bound), float(np.nanmax(err - bound))
        outs.append(got)
        kern.close()
        ctx.close()
    assert np.array_equal(outs[0].view(np.int32), outs[1].view(np.int32))


def test_table_lines_without_or_with_invalid_tile(tmp_path, monkeypatch):
    """A table line without the tile field (the older format), or with a tile the core does not
    take, gives the shape's default tile; the core and block size still come from the line."""
    ctx = apx.Context(0)
    arch = apx.apx_tune_describe(ctx.h).split(",")[0].split()[1]
    ctx.close()
    k = _dev(synth.hann_lowpass(65, 0.3))
    cases = [(f"{arch} 65 {apx.APX_CONV} {apx.APX_ASYM2} 1024 {apx.APX_CORE_INT8} 0 1024 1.000\n", "core=int8", "tiles_per_pass=1"),
             (f"{arch} 65 {apx.APX_CONV} {apx.APX_ASYM2} 1024 {apx.APX_CORE_INT8} 0 1024 1.000 7\n", "core=int8", "tiles_per_pass=1"),
             (f"{arch} 65 {apx.APX_CONV} {apx.APX_ASYM2} 1024 {apx.APX_CORE_TIME} 0 1024 1.000 5\n", "core=time", "outputs_per_thread=4"),
             (f"{arch} 65 {apx.APX_CONV} {apx.APX_ASYM2} 1024 {apx.APX_CORE_TIME} 0 1024 1.000 8\n", "core=time", "outputs_per_thread=8")]
    for i, (line, core, tile) in enumerate(cases):
        path = str(tmp_path / f"t{i}.txt")
        with open(path, "w") as f:
            f.write(line)
        monkeypatch.setenv("APX_TUNE_FILE", path)
        ctx = apx.Context(0)
        kern = apx.Kernel(ctx, k, 1024, mode=apx.APX_ASYM2)
        desc = kern.describe()
        print("case: table line", i, desc, flush=True)
        assert desc.startswith(core) and tile in desc, desc
        kern.close()
        ctx.close()


def test_tune_errors():
    ctx = apx.Context(0)
    with pytest.raises(apx.ApxError) as e:
        apx.apx_tune(ctx.h, _dev(synth.uniform(64, 3)), 1025, apx.params(apx.APX_SYM))  # W odd
    assert e.value.status == apx.APX_E_INVALID
    ctx.close()
