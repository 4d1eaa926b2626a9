"""Seeded synthetic workloads (inputs only; none of the method's arithmetic lives here).

Every generator uses numpy's PCG64 (`numpy.random.default_rng(seed)`) and returns float32
arrays.  Both the tests' oracle side and the HIP side are fed from these functions; the
shapes and value distributions follow the paper's experiments and the measured workloads:

* iid N(0,1) signals and U(-1,1) kernels (plain time-domain case);
* audio-like AR(1) signals (x[t] = a x[t-1] + e[t], e ~ N(0,1)) scaled to [-1, 1];
* Hann-windowed sinc low-pass and band-pass FIR kernels;
* pink (1/f) noise channels;
* U[-128, 128] data as in Section IV.A;
* batched correlation sets (references, noisy template excerpts) and Poisson request streams;
* two-channel audio with a known delay per segment (the multi-channel delay application);
* Weibull-marginal correlated features (the music-matching features of Fig. 4(a)).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.signal import lfilter


def gaussian(L: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(L).astype(np.float32)


def uniform(L: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, L).astype(np.float32)


def ar1(L: int, seed: int, a: float = 0.95) -> np.ndarray:
    """AR(1) driven by unit-variance white noise, scaled by 1/max|x| into [-1, 1]."""
    e = np.random.default_rng(seed).standard_normal(L)
    x = lfilter([1.0], [1.0, -a], e)
    m = np.max(np.abs(x))
    return (x / m).astype(np.float32)


def hann_lowpass(N: int, fc: float = 0.125) -> np.ndarray:
    """Hann-windowed sinc low-pass with cutoff fc (cycles/sample) and unit DC gain."""
    n = np.arange(N) - (N - 1) / 2.0
    h = 2.0 * fc * np.sinc(2.0 * fc * n) * np.hanning(N)
    return (h / np.sum(h)).astype(np.float32)


def hann_bandpass(N: int, f1: float, f2: float) -> np.ndarray:
    """Hann-windowed ideal band-pass [f1, f2] (cycles/sample), peak gain normalised to ~1."""
    n = np.arange(N) - (N - 1) / 2.0
    h = (2.0 * f2 * np.sinc(2.0 * f2 * n) - 2.0 * f1 * np.sinc(2.0 * f1 * n)) * np.hanning(N)
    fc = 0.5 * (f1 + f2)
    g = abs(np.sum(h * np.exp(-2j * np.pi * fc * np.arange(N))))
    return (h / g).astype(np.float32)


def bandpass_bank(n_filters: int = 32, N: int = 512, fmin: float = 0.002, fmax: float = 0.48) -> np.ndarray:
    edges = np.geomspace(fmin, fmax, n_filters + 1)
    return np.stack([hann_bandpass(N, edges[i], edges[i + 1]) for i in range(n_filters)])


def pink_noise(channels: int, L: int, seed: int) -> np.ndarray:
    """1/f noise: Gaussian noise shaped by f^-1/2 in the frequency domain, DC removed, unit RMS."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((channels, L))
    X = np.fft.rfft(x, axis=1)
    f = np.fft.rfftfreq(L)
    g = np.zeros_like(f)
    g[1:] = 1.0 / np.sqrt(f[1:])
    y = np.fft.irfft(X * g, L, axis=1)
    y /= np.sqrt(np.mean(y * y, axis=1, keepdims=True))
    return y.astype(np.float32)


def xcorr_batch(n_templates: int = 4096, n_refs: int = 64, seed_refs: int = 3001, seed_t: int = 3002,
                ref_len=(1 << 18, 1 << 20), tmpl_len=(256, 4096), snr_db: float = 20.0, scale: float = 1.0):
    """References: AR(1) 0.95 signals of lengths U_int[ref_len]; template i is an excerpt of
    reference i mod n_refs at a uniform offset, of length U_int[tmpl_len], plus white noise at
    snr_db.  `scale` < 1 shrinks every length (for small test cases).  Returns
    (refs, templates, ref_index, true_offset)."""
    rng = np.random.default_rng(seed_refs)
    lo, hi = int(ref_len[0] * scale), int(ref_len[1] * scale)
    lens = rng.integers(lo, hi + 1, n_refs)
    refs = [ar1(int(n), seed_refs * 1000 + i) for i, n in enumerate(lens)]
    rt = np.random.default_rng(seed_t)
    tl, th = max(2, int(tmpl_len[0] * scale)), max(2, int(tmpl_len[1] * scale))
    tmpls, ridx, offs = [], [], []
    for i in range(n_templates):
        j = i % n_refs
        n = int(rt.integers(tl, th + 1))
        n = min(n, refs[j].size)
        off = int(rt.integers(0, refs[j].size - n + 1))
        ex = refs[j][off: off + n].astype(np.float64)
        rms = math.sqrt(float(np.mean(ex * ex))) if n else 0.0
        noise = rt.standard_normal(n) * rms * 10.0 ** (-snr_db / 20.0)
        tmpls.append((ex + noise).astype(np.float32))
        ridx.append(j)
        offs.append(off)
    return refs, tmpls, np.array(ridx), np.array(offs)


def weibull_features(L: int, seed: int, lam: float = 0.248, kappa: float = 1.191, a: float = 0.9) -> np.ndarray:
    """Nonnegative, temporally correlated feature sequence with a Weibull(lam, kappa) marginal
    (the music-matching features' fit of Fig. 4(a)): a unit-variance Gaussian AR(1) with
    coefficient a, mapped through the normal CDF and the Weibull inverse CDF."""
    from scipy.special import ndtr
    e = np.random.default_rng(seed).standard_normal(L)
    g = lfilter([math.sqrt(1.0 - a * a)], [1.0, -a], e)
    u = np.clip(ndtr(g), 0.0, 1.0 - 1e-16)
    return (lam * (-np.log1p(-u)) ** (1.0 / kappa)).astype(np.float32)


def two_channel(L: int, seed: int, seg: int = 44100, max_delay: int = 200, mono_frac: float = 0.25,
                snr_db: float = 30.0):
    """Two-channel audio with a known inter-channel delay per segment of `seg` samples.  Channel a
    is AR(1) audio; in a mono segment channel b equals a, in a stereo segment b[n] = a[n - d] with
    1 <= |d| <= max_delay plus white noise at snr_db (zeros before the start of a).  Returns
    (a, b, delays, mono) with one delay and one mono flag per segment."""
    a = ar1(L, seed)
    rng = np.random.default_rng(seed + 1)
    nseg = -(-L // seg)
    mono = rng.random(nseg) < mono_frac
    mag = rng.integers(1, max_delay + 1, nseg)
    delays = np.where(mono, 0, mag * rng.choice([-1, 1], nseg)).astype(np.int64)
    a64 = a.astype(np.float64)
    b = np.empty(L, np.float64)
    for i in range(nseg):
        s0, s1 = i * seg, min(L, (i + 1) * seg)
        d = int(delays[i])
        src = np.arange(s0, s1) - d
        ok = (src >= 0) & (src < L)
        x = np.zeros(s1 - s0)
        x[ok] = a64[src[ok]]
        if not mono[i]:
            rms = math.sqrt(float(np.mean(x * x))) if s1 > s0 else 0.0
            x = x + rng.standard_normal(s1 - s0) * rms * 10.0 ** (-snr_db / 20.0)
        b[s0:s1] = x
    return a, b.astype(np.float32), delays, mono


def poisson_requests(rate: float = 2000.0, duration: float = 10.0, seed: int = 5001,
                     L_range=(1 << 12, 1 << 22), N_range=(16, 4096), n_sizes: int = 32,
                     snr_choices=(30.0, 40.0, 50.0), kernels_per_size: int = 128):
    """Poisson arrivals; L log-uniform, N log-uniform snapped to n_sizes log-spaced values,
    SNR target uniform over snr_choices, kernel index uniform in a pool of kernels_per_size.
    Returns a list of dicts sorted by arrival time."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    sizes = np.unique(np.round(np.geomspace(N_range[0], N_range[1], n_sizes)).astype(int))
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        L = int(round(math.exp(rng.uniform(math.log(L_range[0]), math.log(L_range[1])))))
        N = int(sizes[int(np.argmin(np.abs(np.log(sizes) - rng.uniform(math.log(N_range[0]),
                                                                         math.log(N_range[1])))))])
        out.append({"t": t, "L": L, "N": N, "snr": float(rng.choice(snr_choices)),
                    "seed": int(rng.integers(0, 2 ** 31)), "kernel": int(rng.integers(0, kernels_per_size))})
    return out
