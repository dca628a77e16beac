"""The |V3|^2 model the matrix-free ph-ph path evaluates (rtbte_pp_model)
describes the values the generator stored (CPU only).

Written here from the model's published ingredients, independently of the
generator and of the HIP library: Philox4x32-10 (Salmon, Moraes, Dror and
Shaw, SC'11; checked against its known-answer vectors), the canonical
triplet (sorted ids of the triplet or of its time-reversed image, whichever
is lexicographically smaller), the Box-Muller normal and the lognormal.
Evaluated on a sample of each workload's stored entries, it reproduces the
stored |V3|^2 to rounding.
"""
import math
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
M32 = 0xFFFFFFFF


def philox(ctr, key):
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    for _ in range(10):
        p0 = 0xD2511F53 * c0
        p1 = 0xCD9E8D57 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & M32, p1 & M32, ((p0 >> 32) ^ c3 ^ k1) & M32, p0 & M32
        k0 = (k0 + 0x9E3779B9) & M32
        k1 = (k1 + 0xBB67AE85) & M32
    return c0, c1, c2, c3


def _kat():
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        if line.strip() and not line.startswith("#"):
            w = [int(x, 16) for x in line.split()]
            yield w[:4], w[4:6], w[6:10]


@pytest.mark.parametrize("ctr,key,out", list(_kat()))
def test_philox_known_answers(ctr, key, out):
    assert list(philox(ctr, key)) == out


def reversed_state(i, m):
    nm, L = m["n_modes"], m["L"]
    q, nu = divmod(i, nm)
    if m["dim"] == 2:
        a, b = divmod(q, L)
        nq = ((L - a) % L) * L + (L - b) % L
    else:
        a, r = divmod(q, L * L)
        b, c = divmod(r, L)
        nq = (((L - a) % L) * L + (L - b) % L) * L + (L - c) % L
    return nq * nm + nu


def model_v2(m, l, a, b):
    x = sorted((l, a, b))
    y = sorted(reversed_state(i, m) for i in (l, a, b))
    c = y if y < x else x
    r = philox((c[0], c[1], c[2], m["stream"]), (m["key0"], m["key1"]))
    u1 = (r[1] + 0.5) * 2.0 ** -32
    u2 = (r[2] + 0.5) * 2.0 ** -32
    n = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)
    return math.exp(m["ln_mu"] + m["ln_sigma"] * n)


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "toy2d", "lattice2d"])
def test_model_reproduces_the_stored_values(name):
    wl = synth.build(name)
    if len(wl.pp_row) == 0:
        pytest.skip("no ph-ph entries")
    m = wl.pp_model()
    assert m["n_modes"] * m["L"] ** m["dim"] == wl.n_ph
    rng = np.random.default_rng(11)
    idx = rng.choice(len(wl.pp_row), size=min(2000, len(wl.pp_row)), replace=False)
    got = np.array([model_v2(m, int(wl.pp_row[e]), int(wl.pp_a[e]), int(wl.pp_b[e])) for e in idx])
    assert np.allclose(got, wl.pp_v2[idx], rtol=1e-13, atol=0)


def test_model_symmetries():
    """Permutation and time-reversal invariance, and the distribution: the
    logs of many draws have the model's mean and spread."""
    m = synth.build("tiny2d").pp_model()
    rng = np.random.default_rng(5)
    logs = []
    for _ in range(400):
        l, a, b = (int(v) for v in rng.integers(0, 6 * m["L"] ** 2, 3))
        v = model_v2(m, l, a, b)
        assert v == model_v2(m, b, l, a) == model_v2(m, a, b, l)
        assert v == model_v2(m, reversed_state(l, m), reversed_state(a, m), reversed_state(b, m))
        logs.append(math.log(v))
    logs = np.array(logs)
    assert abs(logs.mean() - m["ln_mu"]) < 4 * m["ln_sigma"] / math.sqrt(len(logs))
    assert abs(logs.std() - m["ln_sigma"]) < 0.15 * m["ln_sigma"]
