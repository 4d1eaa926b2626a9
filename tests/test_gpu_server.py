"""Serving engine (apx_server_*) and the per-call calibrated run (apx_run_auto).

apx_run_auto against the oracle: per-block modes equal the oracle's selection (calibration
measured on block 0, Section IV.D) except at exact ties, packed blocks bit-exact.
Server: every request's output is bit-identical to the same request run alone (apx_run_auto on
its own), whatever the mix, the number of streams or the in-flight limit, and equals the oracle
(packed blocks bit for bit, FP32 blocks within the FP32 bound); the budgeted device memory never
exceeds the budget.
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


@pytest.fixture(scope="module")
def ctx():
    c = apx.Context(0)
    yield c
    c.close()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def _say(*a):
    print(*a, flush=True)


SIZES = [16, 33, 64, 129, 200, 700, 1025, 2000]


def _requests(n, seed, Lmin=4096, Lmax=150000):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        N = SIZES[i % len(SIZES)]
        j = int(rng.integers(0, 3))
        key = N * 10 + j
        k = synth.hann_lowpass(N, 0.05 + 0.1 * j)
        L = int(round(math.exp(rng.uniform(math.log(max(Lmin, N)), math.log(Lmax)))))
        s = synth.ar1(L, seed * 1000 + i)
        op = apx.APX_XCORR if i % 5 == 4 else apx.APX_CONV
        out.append(dict(key=key, k=k, s=s, N=N, L=L, op=op, snr=[30.0, 40.0, 50.0][i % 3]))
    return out


def _serve(ctx, reqs, **cfg):
    srv = apx.Server(ctx, **cfg)
    outs = [np.full(r["L"] + r["N"] - 1, np.nan, np.float32) for r in reqs]
    tickets = [srv.submit(r["key"], r["k"], r["s"], outs[i], r["snr"], op=r["op"]) for i, r in enumerate(reqs)]
    srv.drain()
    comps = {c["ticket"]: c for c in srv.poll(max_n=1024)}
    stats = srv.stats()
    srv.close()
    assert sorted(comps) == sorted(tickets)
    assert all(c["status"] == apx.APX_OK for c in comps.values())
    return outs, [comps[t] for t in tickets], stats


def _alone(ctx, r, W_block, with_info=False):
    kern = apx.Kernel(ctx, _dev(r["k"]), W_block, mode=apx.APX_AUTO_SNR, op=r["op"], snr_min_db=r["snr"])
    ts = _dev(r["s"])
    out = torch.empty(r["L"] + r["N"] - 1, dtype=torch.float32, device=DEV)
    ws = torch.empty(apx.apx_workspace_bytes(), dtype=torch.uint8, device=DEV)
    P = apx.apx_geometry(r["L"], r["N"], W_block)[2]
    info = torch.empty(P * apx.BLOCK_INFO_DTYPE.itemsize, dtype=torch.uint8, device=DEV)
    apx.apx_run_auto(ctx.h, kern.h, ts, out, r["snr"], 0, ws, info)
    torch.cuda.synchronize()
    kern.close()
    if with_info:
        return out.cpu().numpy(), apx.block_info(info)
    return out.cpu().numpy()


def _check_auto_oracle(s, k, op, Wb, snr, got, info):
    """An APX_AUTO_SNR output (calibration on block 0 at S_q = K_q = 8) against the oracle: block
    modes equal the oracle's selection except at exact ties of the model SNR with the target,
    packed blocks bit for bit, FP32 blocks within the FP32 bound.  Returns the calibration and
    the counts (packed, FP32)."""
    kk = k[::-1].copy() if op == apx.APX_XCORR else k
    calib = O.calibrate(s, kk, Wb, block=0, Q=8)
    ps = O.auto_params(s, kk, Wb, snr, calib)
    want = np.array([{O.SYM: 1, O.ASYM2: 2, O.FULL: 0}[p.mode] for p in ps])
    near = np.array([abs(p.snr_pred_db - snr) < 1e-6 for p in ps])
    assert np.array_equal(info["mode"][~near], want[~near])
    packed = (info["mode"] != 0) & ~near
    pred = np.array([p.snr_pred_db for p in ps])
    assert np.allclose(info["snr_pred_db"][packed], pred[packed], rtol=0, atol=1e-6)
    n_packed, n_fp32 = check_mixed_blocks(s, kk, Wb, ps, info["mode"], got, "fft")
    return calib, n_packed, n_fp32


def test_server_mix_equals_alone(ctx):
    reqs = _requests(24, 51)
    _say(f"server: {len(reqs)} requests, L {min(r['L'] for r in reqs)}..{max(r['L'] for r in reqs)}")
    mix, comps, st = _serve(ctx, reqs, hbm_budget=4 << 30, n_streams=4, max_inflight=8)
    _say(f"  stats {st}")
    keys = {(r["key"], r["N"], r["op"]) for r in reqs}
    assert st["kernel_misses"] == len(keys) and st["kernel_hits"] == len(reqs) - len(keys)
    assert st["peak_bytes"] <= 4 << 30
    seq, _, _ = _serve(ctx, reqs, hbm_budget=4 << 30, n_streams=1, max_inflight=1)
    cores = set()
    counts = np.zeros(2, np.int64)
    for i, (r, c) in enumerate(zip(reqs, comps)):
        alone, info = _alone(ctx, r, c["W_block"], with_info=True)
        assert np.array_equal(mix[i].view(np.int32), alone.view(np.int32)), i
        assert np.array_equal(seq[i].view(np.int32), alone.view(np.int32)), i
        # the served output (equal to the alone run) against the oracle
        _, n_packed, n_fp32 = _check_auto_oracle(r["s"], r["k"], r["op"], c["W_block"], r["snr"], mix[i], info)
        counts += (n_packed, n_fp32)
        cores.add(c["core"])
    _say(f"  served outputs equal the oracle: {counts[0]} packed blocks bit for bit, {counts[1]} FP32 blocks in bound")
    assert cores == {apx.APX_CORE_TIME, apx.APX_CORE_FFT}
    assert counts[0] > 0 and counts[1] > 0


@pytest.mark.parametrize("L,N,Wb,snr,op", [(60000, 1024, 4096, 40.0, apx.APX_CONV), (40000, 65, 1024, 30.0, apx.APX_CONV),
                                           (30000, 300, 1024, 50.0, apx.APX_XCORR),
                                           (50000, 129, 1024, 40.0, apx.APX_XCORR)])
def test_run_auto_oracle(ctx, L, N, Wb, snr, op):
    _say(f"run_auto L={L} N={N} W_block={Wb} snr={snr} op={op}")
    s = synth.ar1(L, 700 + N)
    k = synth.hann_lowpass(N, 0.1)
    kern = apx.Kernel(ctx, _dev(k), Wb, mode=apx.APX_AUTO_SNR, op=op, snr_min_db=snr)
    ts = _dev(s)
    ws = torch.empty(apx.apx_workspace_bytes(), dtype=torch.uint8, device=DEV)
    out = torch.empty(L + N - 1, dtype=torch.float32, device=DEV)
    P = apx.apx_geometry(L, N, Wb)[2]
    info = torch.empty(P * apx.BLOCK_INFO_DTYPE.itemsize, dtype=torch.uint8, device=DEV)
    apx.apx_run_auto(ctx.h, kern.h, ts, out, snr, 0, ws, info)
    torch.cuda.synchronize()
    got, info = out.cpu().numpy(), apx.block_info(info)
    kern.close()
    calib, n_packed, n_fp32 = _check_auto_oracle(s, k, op, Wb, snr, got, info)
    _say(f"  calib {calib:.3f} dB, modes {np.bincount(info['mode'], minlength=3)}, {n_fp32} FP32 blocks in bound")


def test_server_budget(ctx):
    budget = 48 << 20
    reqs = []
    for i in range(10):
        N = [65, 1025][i % 2]
        reqs.append(dict(key=N, k=synth.hann_lowpass(N), s=synth.ar1(1 << 20, 90 + i), N=N, L=1 << 20,
                         op=apx.APX_CONV, snr=40.0))
    outs, comps, st = _serve(ctx, reqs, hbm_budget=budget, n_streams=4, max_inflight=16)
    _say(f"  budget {budget}, stats {st}")
    assert st["peak_bytes"] <= budget
    for i in (0, 1, 9):
        assert np.array_equal(outs[i].view(np.int32), _alone(ctx, reqs[i], comps[i]["W_block"]).view(np.int32))
    srv = apx.Server(ctx, hbm_budget=budget, n_streams=2, max_inflight=4)
    big = synth.ar1(1 << 22, 5)
    with pytest.raises(apx.ApxError) as e:
        srv.submit(1, synth.hann_lowpass(65), big, np.empty((1 << 22) + 64, np.float32))
    assert e.value.status == apx.APX_E_NOMEM
    with pytest.raises(apx.ApxError) as e:
        srv.submit(1, synth.hann_lowpass(65), big[:10], np.empty(100, np.float32))
    assert e.value.status == apx.APX_E_INVALID
    assert srv.stats()["rejected"] == 1
    srv.close()


def test_server_batches_requests_of_one_kernel(ctx):
    """Requests that share a prepared kernel and are admitted together run as one launch: a burst
    of 40 requests over 2 kernels behind a long first request comes back in fewer launches than
    requests, every output equal to the request run alone and to the oracle."""
    N = 300
    ks = [synth.hann_lowpass(N, 0.07), synth.hann_lowpass(N, 0.21)]
    reqs = [dict(key=7, k=ks[0], s=synth.ar1(1 << 21, 40), N=N, L=1 << 21, op=apx.APX_CONV, snr=40.0)]
    rng = np.random.default_rng(41)
    for i in range(40):
        L = int(rng.integers(N, 60000))
        j = i % 2
        reqs.append(dict(key=7 + j, k=ks[j], s=synth.ar1(L, 4100 + i), N=N, L=L,
                         op=apx.APX_XCORR if j else apx.APX_CONV, snr=[30.0, 40.0, 50.0][i % 3]))
    outs, comps, st = _serve(ctx, reqs, hbm_budget=4 << 30, n_streams=4, max_inflight=64)
    _say(f"  stats {st}")
    assert st["launches"] < st["completed"] == len(reqs)
    for i in (0, 1, 2, 17, 40):
        r, c = reqs[i], comps[i]
        alone, info = _alone(ctx, r, c["W_block"], with_info=True)
        assert np.array_equal(outs[i].view(np.int32), alone.view(np.int32)), i
        _check_auto_oracle(r["s"], r["k"], r["op"], c["W_block"], r["snr"], outs[i], info)
    for i in range(len(reqs)):
        if i not in (0, 1, 2, 17, 40):
            assert np.array_equal(outs[i].view(np.int32), _alone(ctx, reqs[i], comps[i]["W_block"]).view(np.int32)), i
