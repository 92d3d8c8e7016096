"""On-device sampler's law, written plainly on the CPU -- TEST INFRASTRUCTURE.

The random inclusion model of Sec. 2 (covered domain eqn. Stoch-decomp,
coefficient eqn. ahm_coef) with unit squares whose centres form a Poisson
point process, restricted to the node lattice as the workloads use it: each
of the n^2 lattice sites is independently a square centre with probability
p = occ_threshold / 2^32 (p = 1 - exp(-mu) for mu = expected centres per
site; the sites then carry independent Poisson(mu) centre counts and only
"at least one" matters for the covered set). A square centred at site s
covers the cells s - side/2 + u, u = 0 .. side-1 in each direction (mod n);
a covered cell takes a_in, the others a_bg.

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), written here from its published
definition. Site s = i n + j of realization r uses word s mod 4 of
Philox4x32-10(counter = (s div 4, r mod 2^32, r div 2^32, 0),
key = (seed mod 2^32, seed div 2^32)); it is occupied iff that word is
below occ_threshold. Every step is integer arithmetic, so a correct device
implementation reproduces these fields bit for bit.

The paper's fixed-count law (exactly L^2 squares) draws its centres from the
same generator with another counter tag (fixed_count_centres).

Pins (tests/test_oracle_sample.py): the generator's published known-answer
vectors; the painting rule against a brute-force double loop; occupancy and
coverage frequencies against p and 1 - (1 - p)^(side^2); the fixed-count
centres by Python-integer arithmetic, their uniformity, and the coverage
1 - (1 - side^2/n^2)^K of the fixed-count law.
"""
import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Philox4x32 with 10 rounds on arrays of counters (uint32-valued), one
    key. Round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 as 64-bit
    products; c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is
    bumped by the Weyl constants (W0, W1) before every round but the first."""
    c = [np.asarray(v, dtype=np.uint64) & _MASK for v in (c0, c1, c2, c3)]
    k = [int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF]
    for rnd in range(10):
        if rnd:
            k = [(k[0] + _W0) & 0xFFFFFFFF, (k[1] + _W1) & 0xFFFFFFFF]
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ np.uint64(k[0])) & _MASK, p1 & _MASK,
             ((p0 >> np.uint64(32)) ^ c[3] ^ np.uint64(k[1])) & _MASK, p0 & _MASK]
    return [v.astype(np.uint32) for v in c]


def occupancy(n: int, seed: int, realization: int, occ_threshold: int) -> np.ndarray:
    """(n, n) bool: lattice sites that are square centres."""
    s = np.arange(n * n, dtype=np.uint64)
    g = s // np.uint64(4)
    r = int(realization)
    words = philox4x32_10(g, np.full_like(g, r & 0xFFFFFFFF), np.full_like(g, (r >> 32) & 0xFFFFFFFF),
                          np.zeros_like(g), seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    w = np.stack(words)                                  # (4, n^2 / 4 ... per site group)
    x = w[(s % np.uint64(4)).astype(np.int64), np.arange(n * n)]
    return (x < np.uint32(occ_threshold)).reshape(n, n)


def paint(occ: np.ndarray, side: int, a_in: float, a_bg: float) -> np.ndarray:
    """Cells covered by a side x side square around any occupied site."""
    cov = np.zeros_like(occ)
    for u in range(side):
        cov |= np.roll(occ, u - side // 2, axis=0)
    cov2 = np.zeros_like(cov)
    for v in range(side):
        cov2 |= np.roll(cov, v - side // 2, axis=1)
    return np.where(cov2, float(a_in), float(a_bg))


def field(n: int, side: int, seed: int, realization: int, occ_threshold: int, a_in: float,
          a_bg: float) -> np.ndarray:
    return paint(occupancy(n, seed, realization, occ_threshold), side, a_in, a_bg)


# The paper's own law (Sec. 2, eqn. Stoch-decomp; Sec. 3.1): exactly K = L^2
# squares per realization, each centred at a grid node drawn uniformly (the
# nodes drawn independently, so two squares may share a centre).
FIXED_TAG = 0x46495843   # fourth counter word of the fixed-count centres


def fixed_count_centres(n: int, K: int, seed: int, realization: int) -> np.ndarray:
    """(K,) linear node indices c = i n + j of the K square centres of a
    realization: centre k takes words 0 and 1 of Philox4x32-10 with counter
    (k, r mod 2^32, r div 2^32, FIXED_TAG) and key (seed mod 2^32,
    seed div 2^32) as the 64-bit v = w0 + 2^32 w1, and c = floor(v n^2 / 2^64)
    (uniform on the n^2 nodes up to a bias below n^2 / 2^64)."""
    k = np.arange(int(K), dtype=np.uint64)
    r = int(realization)
    w = philox4x32_10(k, np.full_like(k, r & 0xFFFFFFFF), np.full_like(k, (r >> 32) & 0xFFFFFFFF),
                      np.full_like(k, FIXED_TAG), seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    out = np.empty(int(K), dtype=np.int64)
    nn = n * n
    for i in range(int(K)):
        v = int(w[0][i]) | (int(w[1][i]) << 32)
        out[i] = (v * nn) >> 64
    return out


def fixed_count_field(n: int, side: int, K: int, seed: int, realization: int, a_in: float,
                      a_bg: float) -> np.ndarray:
    """The field of the fixed-count law: squares of side `side` cells around
    the K centres, painted as :func:`paint` does."""
    occ = np.zeros(n * n, dtype=bool)
    occ[fixed_count_centres(n, K, seed, realization)] = True
    return paint(occ.reshape(n, n), side, a_in, a_bg)
