"""Seeded synthetic workloads shaped like the paper's datasets (Table 2).

This module only draws random inputs; it holds none of the search method's
arithmetic.  Every generator is a Gaussian mixture whose samples are snapped
onto a dyadic grid m * 2**-G (|m| < 2**24), so each value is an exact FP32
number and, for the chosen G and value bound B, every squared L2 distance
between two points is an exact FP64 number:  2G + ceil(log2(d * (2B)**2)) <= 53.
That makes FP64 distance sums independent of summation order, which is what
lets a CPU oracle and a GPU kernel agree bit for bit.

Workloads (names used throughout the package):

* ``tiny``      N=10,000, d=32, 16 components, means ~ U[-5,5], sigma=1,
                clipped to [-16,16), grid 2**-19; 100 queries.
* ``sift1m``    N=1,000,000, d=128, 256 components, means ~ U[0,255],
                sigma=20, rounded and clipped to integers 0..255 (grid 2**0);
                10,000 queries and 100,000 training queries.
* ``shift1m``   N=1,000,000, d=96, 512 components, means ~ U[-5,5], sigma=1,
                unit-normalised, grid 2**-22.  Queries (test and training)
                come from the same components with means shifted by
                +0.3*sigma*s_c (s_c a random sign vector per component) and
                Dirichlet(0.3) component weights.
* ``gist1m``    N=1,000,000, d=960, 256 components, x = a * (mu_c + z) with
                a_j ~ LogNormal(0, 0.5), clipped to [-64,64), grid 2**-14;
                1,000 queries, half in-distribution and half mean-shifted.
* ``sift10m``   the ``sift1m`` generator at N=10,000,000 (serving workload),
                30% of queries mean-shifted.

Seeds: master = 250615986 + 1000 * config number, with an independent
substream per role (means, base, queries, train, init, shuffle, weights).
"""
from __future__ import annotations

import dataclasses
import numpy as np

MASTER_SEED = 250615986

ROLES = {"means": 1, "base": 2, "queries": 3, "train": 4, "init": 5,
         "shuffle": 6, "weights": 7, "shift": 8, "scale": 9, "tower": 10,
         "arrivals": 11}


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    config_no: int
    n: int
    d: int
    n_components: int
    n_queries: int
    n_train: int
    grid_exp: int          # G: values are m * 2**-G
    bound: float           # |x| < bound after clipping (or 0..255 for ints)
    kind: str              # "gauss" | "uint8" | "sphere" | "scaled"
    sigma: float
    mean_lo: float
    mean_hi: float
    shift: float = 0.0     # query mean shift in units of sigma
    shifted_frac: float = 0.0
    dirichlet: float = 0.0


WORKLOADS = {
    "tiny": Workload("tiny", 1, 10_000, 32, 16, 100, 1_000, 19, 16.0, "gauss",
                     1.0, -5.0, 5.0),
    "sift1m": Workload("sift1m", 2, 1_000_000, 128, 256, 10_000, 100_000, 0,
                       256.0, "uint8", 20.0, 0.0, 255.0),
    "shift1m": Workload("shift1m", 3, 1_000_000, 96, 512, 10_000, 100_000, 22,
                        1.0, "sphere", 1.0, -5.0, 5.0, shift=0.3,
                        shifted_frac=1.0, dirichlet=0.3),
    "gist1m": Workload("gist1m", 4, 1_000_000, 960, 256, 1_000, 100_000, 14,
                       64.0, "scaled", 1.0, -5.0, 5.0, shift=0.3,
                       shifted_frac=0.5),
    "sift10m": Workload("sift10m", 5, 10_000_000, 128, 256, 10_000, 100_000, 0,
                        256.0, "uint8", 20.0, 0.0, 255.0, shift=0.3,
                        shifted_frac=0.3),
}


def rng_for(w: Workload, role: str, salt: int = 0) -> np.random.Generator:
    master = MASTER_SEED + 1000 * w.config_no
    ss = np.random.SeedSequence([master, ROLES[role], salt])
    return np.random.Generator(np.random.PCG64(ss))


def scaled(w: Workload, n: int | None = None, n_queries: int | None = None,
           n_train: int | None = None) -> Workload:
    """Same recipe with different counts (parity cases at reduced N)."""
    return dataclasses.replace(
        w, n=w.n if n is None else n,
        n_queries=w.n_queries if n_queries is None else n_queries,
        n_train=w.n_train if n_train is None else n_train)


def _snap(x: np.ndarray, w: Workload) -> np.ndarray:
    if w.kind == "uint8":
        return np.clip(np.rint(x), 0.0, 255.0).astype(np.float32)
    scale = float(2 ** w.grid_exp)
    lim = w.bound * scale
    m = np.clip(np.rint(x * scale), -lim, lim - 1)
    return (m / scale).astype(np.float32)


def _means(w: Workload) -> np.ndarray:
    r = rng_for(w, "means")
    return r.uniform(w.mean_lo, w.mean_hi, size=(w.n_components, w.d))


def _scale_vec(w: Workload) -> np.ndarray | None:
    if w.kind != "scaled":
        return None
    return rng_for(w, "scale").lognormal(0.0, 0.5, size=w.d)


def _shift_signs(w: Workload) -> np.ndarray:
    r = rng_for(w, "shift")
    return r.choice(np.array([-1.0, 1.0]), size=(w.n_components, w.d))


def _draw(w: Workload, n: int, role: str, salt: int, shifted: np.ndarray | None,
          weights: np.ndarray | None, chunk: int = 1 << 18) -> np.ndarray:
    """n samples; shifted[i] says whether sample i uses the shifted means."""
    mu = _means(w)
    a = _scale_vec(w)
    s = _shift_signs(w) if shifted is not None else None
    r = rng_for(w, role, salt)
    if weights is None:
        comp = r.integers(0, w.n_components, size=n)
    else:
        comp = r.choice(w.n_components, size=n, p=weights)
    out = np.empty((n, w.d), dtype=np.float32)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        c = comp[lo:hi]
        m = mu[c]
        if s is not None:
            sh = shifted[lo:hi, None]
            m = m + np.where(sh, w.shift * w.sigma * s[c], 0.0)
        x = m + w.sigma * r.standard_normal((hi - lo, w.d))
        if w.kind == "sphere":
            x /= np.linalg.norm(x, axis=1, keepdims=True)
        elif w.kind == "scaled":
            x *= a[None, :]
        out[lo:hi] = _snap(x, w)
    return out


def base(w: Workload) -> np.ndarray:
    """N x d float32 base vectors (row-major)."""
    return _draw(w, w.n, "base", 0, None, None)


def _query_mix(w: Workload, n: int, role: str, salt: int):
    r = rng_for(w, role, 1000 + salt)
    shifted = r.random(n) < w.shifted_frac if w.shifted_frac > 0 else None
    weights = None
    if w.dirichlet > 0:
        weights = rng_for(w, "weights").dirichlet(
            np.full(w.n_components, w.dirichlet))
    return shifted, weights


def queries(w: Workload, n: int | None = None) -> np.ndarray:
    """Test queries."""
    n = w.n_queries if n is None else n
    shifted, weights = _query_mix(w, n, "queries", 0)
    return _draw(w, n, "queries", 0, shifted, weights)


def train_queries(w: Workload, n: int | None = None) -> np.ndarray:
    """Historical (training) queries, drawn like the test queries."""
    n = w.n_train if n is None else n
    shifted, weights = _query_mix(w, n, "train", 0)
    return _draw(w, n, "train", 0, shifted, weights)


def kmeans_init(w: Workload, n: int, n_hubs: int) -> np.ndarray:
    """First n_hubs entries of a seeded permutation of range(n) (int32)."""
    return rng_for(w, "init").permutation(n)[:n_hubs].astype(np.int32)


def tower_init(w: Workload, shapes: list[tuple[int, int]], salt: int = 0) -> list[np.ndarray]:
    """Uniform(-1/sqrt(fan_in), +1/sqrt(fan_in)) weights/biases, float32.

    shapes are (out, in) per linear layer; returns [W0, b0, W1, b1, ...].
    salt picks an independent substream (0: the towers')."""
    r = rng_for(w, "tower", salt)
    out = []
    for (o, i) in shapes:
        lim = 1.0 / np.sqrt(i)
        out.append(r.uniform(-lim, lim, size=(o, i)).astype(np.float32))
        out.append(r.uniform(-lim, lim, size=(o,)).astype(np.float32))
    return out


def batch_order(w: Workload, n: int, epoch: int) -> np.ndarray:
    """Seeded shuffle of training-query indices for one epoch."""
    return rng_for(w, "shuffle", epoch).permutation(n).astype(np.int64)


def queue_batch(w: Workload, step: int, eligible: np.ndarray, pos_off: np.ndarray,
                neg_off: np.ndarray, hubs: int, P: int, N: int):
    """Seeded choice for one hub-anchored training step: `hubs` hubs drawn
    without replacement from `eligible`, and for each P positions into its
    positive queue and N into its negative queue, with replacement (queue h
    spans off[h] .. off[h+1] of the concatenated queues).  Returns (hub
    indices [b], positive positions [b, P], negative positions [b, N])."""
    r = rng_for(w, "shuffle", 1_000_000 + step)
    hb = r.choice(eligible, size=min(hubs, eligible.size), replace=False).astype(np.int64)
    pp = np.empty((hb.size, P), np.int64)
    nn = np.empty((hb.size, N), np.int64)
    for i, h in enumerate(hb):
        pp[i] = pos_off[h] + r.integers(0, pos_off[h + 1] - pos_off[h], size=P)
        nn[i] = neg_off[h] + r.integers(0, neg_off[h + 1] - neg_off[h], size=N)
    return hb, pp, nn


def request_stream(w: Workload, n_requests: int, rate: float, max_batch: int = 512):
    """Poisson arrivals: (arrival_s, batch_size, k) per request."""
    r = rng_for(w, "arrivals")
    gaps = r.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    sizes = r.integers(1, max_batch + 1, size=n_requests)
    ks = np.where(r.random(n_requests) < 0.5, 10, 100)
    return t, sizes.astype(np.int64), ks.astype(np.int32)
