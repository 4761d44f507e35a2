"""The deposit entry point that allocates nothing (hp_debug_deposit_noalloc,
for callers that cannot allocate device memory) against hp_debug_deposit, the
entry point it is a variant of: the same 64-bit accumulators bit for bit, on
two calls in a row (the second with fewer moves and a smaller grid, so the
region still holds the first call's larger contents), and sizes beyond the
region rejected with HP_EINVAL."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MAX_MOVES = 1 << 18


def _moves(n1, n2, npart, seed):
    gen = np.random.default_rng(seed)
    c0 = np.stack([gen.integers(0, n1, npart), gen.integers(0, n2, npart)]).astype(np.int32)
    o0 = gen.random((2, npart)).astype(np.float32)
    x1 = c0 + o0.astype(np.float64) + gen.uniform(-0.99, 0.99, (2, npart))
    c1 = np.floor(x1).astype(np.int64)
    o1 = (x1 - c1).astype(np.float32)
    over = o1 >= 1
    c1[over] += 1
    o1[over] = 0
    c1[0] %= n1
    c1[1] %= n2
    v3 = gen.uniform(-0.95, 0.95, npart).astype(np.float32)
    qw = gen.uniform(-1.0, -0.5, npart).astype(np.float32)
    return c0, o0, c1.astype(np.int32), o1, v3, qw


def _sim(hpic, n1, n2, seed):
    sim = hpic.Sim([hpic.config(n1, n2, 0.1, 0.2, 0.045)])
    gen = np.random.default_rng(seed)
    xi = np.stack([gen.uniform(0, n1, 500), gen.uniform(0, n2, 500)])
    sim.set_particles(0, xi * np.array([[0.1], [0.2]]), np.zeros((3, 500)),
                      gen.uniform(0.5, 1.0, 500), -1.0, -1.0)
    return sim


def test_noalloc_deposit_equals_allocating_deposit(hpic):
    for (n1, n2, npart, seed) in ((512, 256, 200000, 7), (64, 32, 3000, 8)):
        sim = _sim(hpic, n1, n2, seed)
        mv = _moves(n1, n2, npart, seed + 100)
        want = sim.debug_deposit(0, *mv)
        got = sim.debug_deposit(0, *mv, noalloc=True)
        assert np.array_equal(got, want)
        assert np.abs(want).max() > 0
        sim.close()


def test_noalloc_deposit_limits(hpic):
    sim = _sim(hpic, 64, 32, 9)
    n = MAX_MOVES + 1
    mv = _moves(64, 32, n, 10)
    with pytest.raises(hpic.HpError) as e:
        sim.debug_deposit(0, *mv, noalloc=True)
    assert e.value.code == hpic.HP_EINVAL
    sim.close()
    big = _sim(hpic, 1024, 512, 11)  # 524288 cells > 262144
    mv = _moves(1024, 512, 100, 12)
    with pytest.raises(hpic.HpError) as e:
        big.debug_deposit(0, *mv, noalloc=True)
    assert e.value.code == hpic.HP_EINVAL
    # the allocating entry point still takes it
    assert np.abs(big.debug_deposit(0, *mv)).max() > 0
    big.close()
