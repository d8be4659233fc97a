"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds input generation only and none of the evolution arithmetic.

Initial field (the paper generates its "numerical" initial conditions once, in
single precision, and feeds the same field to every run, Sec. III): every site
draws an independent value uniform on the open interval (-1, 1) from a
counter-based generator, so the value depends only on (seed, site index) and
never on how the lattice is split:

    z_i   = SplitMix64 output for counter i + 1 under the given seed
            (Steele, Lea & Flood, "Fast splittable pseudorandom number
            generators", OOPSLA 2014: state += 0x9E3779B97F4A7C15, then the
            variant-13 finaliser with shifts 30/27/31 and multipliers
            0xBF58476D1CE4E5B9, 0x94D049BB133111EB)
    k_i   = top 24 bits of z_i
    phi_i = (2 k_i + 1) / 2^24 - 1

Each value is an odd multiple of 2^-24 in (-1, 1): exact in float32, never 0
and symmetric about 0.  The initial field derivative is 0.
"""
import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, counter):
    """SplitMix64 output for the given counter values (uint64 array, 1-based
    counters as in the published generator's first call)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + np.asarray(counter, dtype=np.uint64) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_sites(seed, start, count):
    """float32 values of sites start .. start+count-1 (linear index)."""
    idx = np.arange(start, start + count, dtype=np.uint64) + np.uint64(1)
    k = (splitmix64(seed, idx) >> np.uint64(40)).astype(np.int64)
    # (2k+1)/2^24 - 1 == (2k + 1 - 2^24) / 2^24, exact in float32
    return ((2 * k + 1 - (1 << 24)).astype(np.float32) * np.float32(2.0 ** -24))


def uniform_field(shape, seed, chunk=1 << 24):
    """Initial field of the given lattice shape (nx, ny[, nz]) as a float32
    array in site order i = x + nx*(y + ny*z), i.e. numpy shape reversed."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        out[s:e] = uniform_sites(seed, s, e - s)
    return out.reshape(tuple(reversed(shape)))


def ensemble_draw(master_seed=2017, n2d=48, n3d=16,
                  sizes2d=(512, 1024, 2048), sizes3d=(128, 256),
                  eras=(0.5, 1.0, 2.0), widths=(5.0, 10.0)):
    """Realisation list of the batched-ensemble workload: sizes, expansion
    rates m and wall widths W0 drawn uniformly from the given sets by a numpy
    generator seeded with master_seed; realisation r gets field seed 1000 + r
    and runs to eta = N/2 (deta 0.25 in 2D, 0.2 in 3D, eta0 = 1)."""
    rng = np.random.default_rng(master_seed)
    items = []
    for r in range(n2d + n3d):
        three = r >= n2d
        sizes = sizes3d if three else sizes2d
        N = int(sizes[rng.integers(len(sizes))])
        m = float(eras[rng.integers(len(eras))])
        W0 = float(widths[rng.integers(len(widths))])
        deta = 0.2 if three else 0.25
        eta_end = N / 2.0
        steps = int(round((eta_end - 1.0) / deta))
        items.append({"ndim": 3 if three else 2, "N": N, "m": m, "W0": W0,
                      "deta": deta, "steps": steps, "seed": 1000 + r})
    return items


def uniform_at(seed, index):
    """float32 initial-field values at arbitrary linear site indices."""
    idx = np.asarray(index, dtype=np.uint64) + np.uint64(1)
    k = (splitmix64(seed, idx) >> np.uint64(40)).astype(np.int64)
    return ((2 * k + 1 - (1 << 24)).astype(np.float32) * np.float32(2.0 ** -24))
