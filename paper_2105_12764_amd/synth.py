"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module draws coordinates and fields only; it holds none of the
refactoring arithmetic, so both the HIP library's callers and the CPU oracle's
callers can use it without sharing method code.

The paper evaluates on Gray-Scott reaction-diffusion outputs (Sec. IV-A) and
notes that the running time does not depend on the values, only on the grid
size.  Those outputs are not available, so smooth multi-frequency fields with
a small noise floor stand in for them:

* coordinates per dimension, drawn first, dimension 0 first: uniform
  ``x_i = i``, or non-uniform ``x_0 = 0, x_{i+1} = x_i + U[0.5, 1.5]``;
* normalised position ``t_k = (x - x_0) / (x_{n-1} - x_0)``;
* four sinusoids with integer frequency vectors in ``{1..8}^d`` and phases in
  ``[0, 2 pi)``, amplitude 1, plus N(0, sigma = 1e-3) noise drawn in C order;
* FP32 fields are drawn in FP64 and then rounded.
"""
from __future__ import annotations

import numpy as np

N_WAVES = 4
NOISE_SIGMA = 1e-3


def make_coords(shape, rng: np.random.Generator, nonuniform: bool):
    """Per-dimension strictly increasing FP64 coordinates."""
    out = []
    for n in shape:
        if nonuniform:
            x = np.empty(n, dtype=np.float64)
            x[0] = 0.0
            if n > 1:
                x[1:] = np.cumsum(rng.uniform(0.5, 1.5, size=n - 1))
        else:
            x = np.arange(n, dtype=np.float64)
        out.append(x)
    return out


def make_field(shape, coords, rng: np.random.Generator) -> np.ndarray:
    """Sum of seeded sinusoids plus Gaussian noise, FP64, C order."""
    d = len(shape)
    freqs = rng.integers(1, 9, size=(N_WAVES, d))
    phases = rng.uniform(0.0, 2.0 * np.pi, size=N_WAVES)
    ts = [(c - c[0]) / (c[-1] - c[0]) for c in coords]
    # sin(2 pi f.t + phi) = Im(e^{i phi} prod_k e^{i 2 pi f_k t_k}); the
    # product form builds the field from 1-D factors without a 3-D sin.
    acc = np.zeros(shape, dtype=np.complex128)
    for j in range(N_WAVES):
        term = np.exp(1j * phases[j]) * np.ones((), dtype=np.complex128)
        factor = None
        for k in range(d):
            e = np.exp(2j * np.pi * freqs[j, k] * ts[k])
            sh = [1] * d
            sh[k] = shape[k]
            e = e.reshape(sh)
            factor = e if factor is None else factor * e
        acc += term * factor
    u = acc.imag
    del acc
    u += rng.normal(0.0, NOISE_SIGMA, size=shape)
    return np.ascontiguousarray(u)


def make_input(shape, seed: int, nonuniform: bool = False, dtype=np.float64):
    """(field, coords) for one seeded case; coords is None when uniform."""
    rng = np.random.default_rng(seed)
    coords = make_coords(shape, rng, nonuniform)
    u = make_field(shape, coords, rng)
    if dtype == np.float32:
        u = u.astype(np.float32)
    return u, (coords if nonuniform else None)


# Named workloads: (shape, seed, nonuniform coordinates, dtype, level count)
WORKLOADS = {
    "cube65_f64": ((65, 65, 65), 1001, False, np.float64, 5),
    "cube513_f64": ((513, 513, 513), 1002, False, np.float64, 9),
    "cube513_f32": ((513, 513, 513), 1002, False, np.float32, 9),
    "box400x300x250_f32": ((400, 300, 250), 1003, True, np.float32, 8),
}


def batch_specs(nfields: int = 64, seed0: int = 4000):
    """Shapes and dtypes of the mixed batch: field i draws, from its own
    generator seeded (seed0, i), a rank of 2 or 3 (probability 1/2 each), FP32
    or FP64 (1/2 each) and a side length log-uniform over [257, 2049] (2-D) or
    [33, 257] (3-D); its values come from make_input with seed seed0 + i.
    Returns [(shape, dtype, seed)]."""
    out = []
    for i in range(nfields):
        rng = np.random.default_rng([seed0, i])
        dim = 2 if rng.random() < 0.5 else 3
        dtype = np.float32 if rng.random() < 0.5 else np.float64
        lo, hi = (257, 2049) if dim == 2 else (33, 257)
        side = int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))
        out.append(((side,) * dim, dtype, seed0 + i))
    return out


# Cube sides of the service workload: integers, log-uniform over [17, 513].
SERVICE_SIDE_MIN, SERVICE_SIDE_MAX = 17, 513


def service_requests(nreq: int, seed: int = 5000):
    """The request stream of the service workload: request i has a 3-D cube
    side round(exp(U[log 17, log 513])) (an integer, log-uniform over
    [17, 513]), FP32 with probability 3/4 (else FP64), recompose with
    probability 1/2 (else decompose), and a unit-rate exponential gap before
    its arrival (divide the running sum by the arrival rate for Poisson
    arrivals).  Returns [(side, dtype, recompose, gap)]."""
    rng = np.random.default_rng(seed)
    sides = np.rint(np.exp(rng.uniform(np.log(SERVICE_SIDE_MIN), np.log(SERVICE_SIDE_MAX), size=nreq)))
    sides = np.clip(sides, SERVICE_SIDE_MIN, SERVICE_SIDE_MAX).astype(int)
    fp32 = rng.random(nreq) < 0.75
    rec = rng.random(nreq) < 0.5
    gaps = rng.exponential(1.0, size=nreq)
    return [(int(s), np.float32 if f else np.float64, bool(r), float(g))
            for s, f, r, g in zip(sides, fp32, rec, gaps)]
