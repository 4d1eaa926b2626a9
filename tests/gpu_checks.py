"""Checks shared by the GPU parity tests: error bounds of the FP32 paths and the comparison of a
mixed-mode (per-block choice) output with the oracle.  Test infrastructure: calls the oracle and
numpy only.
"""
import math

import numpy as np

import oracle as O

# apx_mode of a block report -> the oracle's mode name
MODE_OF = {1: O.SYM, 2: O.ASYM2, 3: O.ASYM3, 0: O.FULL}


def fp32_bound(s, k, Wb, core):
    """Per-output bound on |r_fp32 - r_fp64|.  Time domain: sequential FMA sums of N terms,
    |err| <= 2 N u (|s| * |k|)[m] with u = 2^-24.  FFT core (length F, radix-8 Stockham):
    |err| <= 8 log2(F) u ||x_block||_2 ||k||_2 + 2 N u (|s| * |k|)[m] as a generous normwise bound."""
    u = 2.0 ** -24
    N = len(k)
    absconv = O.conv_direct(np.abs(s.astype(np.float64)), np.abs(k.astype(np.float64)))
    b = 2.0 * N * u * absconv + 1e-30
    if core == "fft":
        part = O.partition(len(s), N, Wb)
        F = max(2048, 1 << int(math.ceil(math.log2(2 * Wb))))   # largest transform either core uses
        kn = float(np.linalg.norm(k.astype(np.float64)))
        for w in range(part.P):
            j_lo, j_hi, o = part.keep(w)
            xn = float(np.linalg.norm(part.window(s, w).astype(np.float64)))
            b[o: o + j_hi - j_lo] += 8.0 * math.log2(F) * u * xn * kn
    return b


def check_mixed_blocks(s, k, Wb, ps, modes, got, core="fft", ref64=None):
    """Outputs of a run whose blocks each took their own mode (block report `modes`, apx_mode
    values) against the oracle: blocks in a packed mode equal the plain definition bit for bit
    (conv_blocked with that block's companding); blocks in full precision (FP32) lie within
    fp32_bound of the FP64 direct convolution.  `ps` are the oracle's BlockParams for the same
    blocks (their S, K as the selection gave them); their modes are set from `modes` here.
    Returns (number of packed blocks, number of FP32 blocks)."""
    modes = np.asarray(modes)
    for p, m in zip(ps, modes):
        p.mode = MODE_OF[int(m)]
    ref = O.conv_blocked(s, k, Wb, ps)
    part = O.partition(len(s), len(k), Wb)
    assert modes.size == part.P
    full = modes == 0
    bound = None
    if full.any():
        if ref64 is None:
            ref64 = O.conv_direct(s, k)
        bound = fp32_bound(s, k, Wb, core)
    for w in range(part.P):
        j_lo, j_hi, o = part.keep(w)
        sl = slice(o, o + j_hi - j_lo)
        if modes[w] != 0:
            bad = np.nonzero(got[sl].view(np.int32) != ref[sl].view(np.int32))[0]  # bit for bit
            assert bad.size == 0, f"block {w} (mode {modes[w]}): {bad.size} outputs differ, first at {o + bad[:4]}"
        else:
            err = np.abs(got[sl].astype(np.float64) - ref64[sl])
            over = np.nonzero(~(err <= bound[sl]))[0]
            assert over.size == 0, \
                f"FP32 block {w}: {over.size} outputs beyond the FP32 bound, worst {float(np.nanmax(err))}"
    return int(np.count_nonzero(~full)), int(np.count_nonzero(full))
