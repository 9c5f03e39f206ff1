"""Seeded draws for keys, ciphertexts, tables and request traces.

Every function here returns plain numpy arrays sampled from a numpy
``Generator`` keyed by ``(seed, stream tag)``.  Nothing here combines the
draws: the phase, the gadget, the key layout and the test vector are built by
the two implementations separately.

Distributions
-------------
* uniform residues in [0, M) for key masks and encryption masks;
* binary secrets s in {0,1}^n and z in {0,1}^N (the secret distribution of the
  single-key CMux with d_- = 0, Sec. 2 item (15)), or a ternary s in {-1,0,1}^n
  (Alg. 1 as printed, two keys per coordinate);
* the discrete Gaussian on Z with P(x) proportional to exp(-x^2 / (2 sigma^2)),
  tail-cut at 12 sigma, for every error term (sigma = 0 gives the noise-free
  mode used for end-to-end correctness at large t);
* look-up tables: f(m) uniform on [0, t') for m < t/2 and extended by
  f(m + t/2) = -f(m) mod t', so that f is nega-cyclic (Sec. 2 item (7),
  Definition 1).
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

# 2^31 - 2^17 + 1: prime, = 1 mod 2^17, so it carries negacyclic NTTs of every
# power-of-two degree up to 2^16.
Q_DEFAULT = 2147352577
# 2^23 - 2^13 + 1: prime, = 1 mod 2^13; with Q_DEFAULT a ring modulus of 54 bits
# for negacyclic NTTs up to degree 4096.
Q2_DEFAULT = 8380417

_TAGS = {
    "s": 1, "z": 2, "bsk_a": 3, "bsk_e": 4, "ksk_a": 5, "ksk_e": 6,
    "enc_a": 7, "enc_e": 8, "msg": 9, "table": 10, "mix": 11, "arrivals": 12,
}


def _rng(seed: int, tag: str) -> np.random.Generator:
    return np.random.default_rng([int(seed) & 0xFFFFFFFFFFFFFFFF, _TAGS[tag]])


def _uniform_u32(seed: int, tag: str, bound: int, shape) -> np.ndarray:
    """Uniform uint32 in [0, bound).  Arrays of 2^30 words or more (the
    key-switching masks of the largest rings) are drawn in 64 blocks along the
    first axis, each from its own stream spawned off the same (seed, tag), on
    several threads; smaller arrays come from the one stream of (seed, tag)."""
    if int(np.prod(shape)) < (1 << 30):
        return _rng(seed, tag).integers(0, bound, size=shape, dtype=np.uint32)
    import os
    from concurrent.futures import ThreadPoolExecutor
    out = np.empty(shape, dtype=np.uint32)
    blocks = 64
    kids = np.random.SeedSequence([int(seed) & 0xFFFFFFFFFFFFFFFF, _TAGS[tag]]).spawn(blocks)
    edges = np.linspace(0, shape[0], blocks + 1).astype(np.int64)

    def fill(b):
        g = np.random.Generator(np.random.PCG64(kids[b]))
        lo, hi = int(edges[b]), int(edges[b + 1])
        out[lo:hi] = g.integers(0, bound, size=(hi - lo,) + tuple(shape[1:]), dtype=np.uint32)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(fill, range(blocks)))
    return out


@dataclass(frozen=True)
class Params:
    """Ring and gadget parameters shared by every table of one key set."""

    n: int            # LWE dimension
    N: int            # ring degree (power of two)
    Q: int = Q_DEFAULT
    log2_B: int = 7   # blind-rotation gadget base 2^log2_B
    l: int = 4        # blind-rotation gadget length
    log2_Bks: int = 4  # key-switch base 2^log2_Bks
    l_ks: int = 8     # key-switch length (ceil(31 / log2_Bks) makes it exact)
    sigma: float = 3.2
    sigma_ks: float = 3.2
    ternary: bool = False  # s in {-1, 0, 1}^n with two RGSW keys per coordinate
    Q2: int = 0       # nonzero: the blind rotation runs at the ring modulus Q * Q2

    @property
    def B_ks(self) -> int:
        return 1 << self.log2_Bks

    @property
    def Q_ring(self) -> int:
        """Modulus of the accumulator and of the bootstrapping key."""
        return self.Q * self.Q2 if self.Q2 else self.Q

    @property
    def keys_per_coord(self) -> int:
        return 2 if self.ternary else 1

    def noise_free(self) -> "Params":
        return replace(self, sigma=0.0, sigma_ks=0.0)


# Named workloads.  "tiny": n=64, N=256, k=2, t=16, base 2^8 x 3.
# "paper_shaped": n=630, N=1024, k=4, t=2^12, base 2^7 x 4, key switch 2^4 x 8.
# "tfhe_shaped": the same t = 2^12 by one ring of degree N k = 4096 (r = 1),
# the TFHE side of the comparison in Sec. 5.
PRESETS = {
    "tiny": dict(params=Params(n=64, N=256, log2_B=8, l=3), t=16, t_out=16, r=2),
    "paper_shaped": dict(params=Params(n=630, N=1024, log2_B=7, l=4), t=4096, t_out=4096, r=4),
    "tfhe_shaped": dict(params=Params(n=630, N=4096, log2_B=7, l=4), t=4096, t_out=4096, r=1),
    # The parameters of the experiments in Sec. 5: log n = 9, log N = 11, a ring
    # modulus of 54 bits (2147352577 x 8380417), gadget 2^15 x 4, a ternary secret
    # (two RGSW keys per coordinate), q = 2Nr with 2Nr / t = 128 (so r = t / 32,
    # log r = log t - 5 as in Tables 1-2); t = 2^12 needs r = 128.
    "paper_margin": dict(params=Params(n=512, N=2048, log2_B=15, l=4, Q2=Q2_DEFAULT, ternary=True), t=4096,
                         t_out=4096, r=128),
}

# (t, r) classes of the uneven batch and of the serving trace: q = 2Nr each.
CLASS_MIX = ((256, 1), (1024, 2), (4096, 4), (16384, 8))


def discrete_gaussian(rng: np.random.Generator, sigma: float, size) -> np.ndarray:
    """Discrete Gaussian on Z (tail-cut at 12 sigma) as int32."""
    if sigma == 0:
        return np.zeros(size, dtype=np.int32)
    tail = int(np.ceil(12 * sigma))
    support = np.arange(-tail, tail + 1, dtype=np.int64)
    w = np.exp(-(support.astype(np.float64) ** 2) / (2.0 * sigma * sigma))
    idx = rng.choice(support.size, size=size, p=w / w.sum())
    return support[idx].astype(np.int32)


def key_draws(p: Params, seed: int) -> dict:
    """All random material of one key set.

    Shapes: s (n,) int32, z (N,), bsk_a (n * K, 2l, N) (uint64 in [0, Q Q2) when Q2
    is set), bsk_e (n * K, 2l, N) with K
    keys per coordinate (1 binary, 2 ternary; key k of coordinate i at row i K + k),
    ksk_a (N, l_ks, B_ks, n), ksk_e (N, l_ks, B_ks).
    """
    n, N, l, Q = p.n, p.N, p.l, p.Q
    K = p.keys_per_coord
    lo = -1 if p.ternary else 0
    out = {
        "s": _rng(seed, "s").integers(lo, 2, size=n).astype(np.int32),
        "z": _rng(seed, "z").integers(0, 2, size=N, dtype=np.uint32),
        "bsk_a": _rng(seed, "bsk_a").integers(0, p.Q_ring, size=(n * K, 2 * l, N),
                                              dtype=np.uint64 if p.Q2 else np.uint32),
        "bsk_e": discrete_gaussian(_rng(seed, "bsk_e"), p.sigma, (n * K, 2 * l, N)),
        "ksk_a": _uniform_u32(seed, "ksk_a", Q, (N, p.l_ks, p.B_ks, n)),
        "ksk_e": discrete_gaussian(_rng(seed, "ksk_e"), p.sigma_ks, (N, p.l_ks, p.B_ks)),
    }
    return out


def enc_draws(n: int, q: int, count: int, seed: int, sigma: float = 3.2) -> dict:
    """Masks a (count, n) uniform in [0, q) and errors e (count,)."""
    return {
        "a": _rng(seed, "enc_a").integers(0, q, size=(count, n), dtype=np.uint32),
        "e": discrete_gaussian(_rng(seed, "enc_e"), sigma, (count,)),
    }


def messages(t: int, count: int, seed: int) -> np.ndarray:
    return _rng(seed, "msg").integers(0, t, size=count, dtype=np.uint32)


def negacyclic_table(t: int, t_out: int, seed: int) -> np.ndarray:
    """Random f: Z_t -> Z_t' with f(m + t/2) = -f(m) mod t'."""
    half = _rng(seed, "table").integers(0, t_out, size=t // 2, dtype=np.int64)
    f = np.concatenate([half, (-half) % t_out])
    return f.astype(np.uint32)


def class_mix(count: int, seed: int, classes=CLASS_MIX) -> np.ndarray:
    """Index into ``classes`` drawn uniformly per ciphertext."""
    return _rng(seed, "mix").integers(0, len(classes), size=count, dtype=np.int32)


def poisson_arrivals(rate_per_s: float, count: int, seed: int) -> np.ndarray:
    """Arrival offsets in nanoseconds of a Poisson process (exponential gaps)."""
    gaps = _rng(seed, "arrivals").exponential(1.0 / rate_per_s, size=count)
    return np.cumsum(gaps * 1e9).astype(np.int64)
