"""Pins of the oracle's triage features (orc_features): small programs whose
128 features are worked out by hand from the feature definition."""
import numpy as np

from oracle import oracle as O


def _expect(entries, shape_part):
    """entries: index -> number, or (num, den) for the fp32 quotient."""
    f = np.zeros(128, dtype=np.float32)
    for d in (entries, shape_part):
        for k, v in d.items():
            f[k] = np.float32(v[0]) / np.float32(v[1]) if isinstance(v, tuple) else np.float32(v)
    return f


def sq(c, k):
    """A bounded count: c / (c + k)."""
    return (c, c + k)


def _hist(values, lo, hi, cells):
    h = np.zeros(8)
    for v in values[:cells]:
        h[(v - lo) * 8 // (hi - lo)] += 1
    return h / 256


SRC1 = """
kernel k(global int A[64], global int B[8]) {
  int v;
  v := A[tid];
  A[(tid + 1) mod 64] := v;
  barrier;
  B[0] := tid;
  if (v < 3) {
    B[2] := 1;
  }
}
"""


def test_features_two_intervals_with_shifted_and_constant_cells():
    p = O.Program(SRC1)
    Bdata = np.array([-2**31, -1, 0, 2**31 - 1, 536870911, 536870912, -536870913, 100], dtype=np.int32)
    G, W, seed = 3, 40, 11
    f = p.features(G, W, {"A": ("seeded", 0, 16), "B": Bdata}, seed=seed)
    # statements in order: load, store, barrier, store, if, store  (6)
    e = {1: (1, 6), 2: (3, 6), 3: (1, 6), 6: (1, 6),
         8: (1, 6), 10: (3, 6), 12: sq(6, 256), 13: (2, 8),
         # self pairs with a constant cell: B[0], B[2] (the second under an if);
         # shifted pairs: A[tid] / A[tid+1 mod 64], B[0] / B[2]
         16: sq(2, 8), 17: sq(1, 8), 19: sq(2, 8),
         24: sq(1, 16), 25: sq(1, 16), 26: sq(1, 16), 28: sq(1, 16), 30: sq(2, 8),
         # of the shifted pairs, A's meet one work-item apart; B[0] / B[2]
         # (a = 0) never do
         31: sq(1, 8),
         # memory statements: (kind, a/(1+|a|), b/size, (interval+1)/8)
         32: -1, 33: 0.5, 34: 0, 35: (1, 8),
         36: 1, 37: 0.5, 38: (1, 64), 39: (1, 8),
         40: 1, 41: 0, 42: 0, 43: (2, 8),
         44: 1, 45: 0, 46: (2, 8), 47: (2, 8),
         96: sq(1, 8), 98: sq(2, 64), 100: sq(4, 64), 101: sq(3, 64), 102: sq(2, 8)}
    shape = {104: (W, 1024), 105: (G, 1024), 106: (6, 32), 107: (3, 32), 109: (G * W, 2**20)}
    want = _expect(e, shape)
    avals = [O.seeded_value(seed, 0, c, 0, 16) for c in range(64)]
    want[112:120] = _hist(avals, 0, 16, 64).astype(np.float32)
    # bound buffer: eighths of the int32 range -> bins 0, 3, 4, 7, 4, 5, 2, 4
    want[120:128] = np.array([1, 0, 1, 1, 3, 1, 0, 1], dtype=np.float32) / 256
    assert np.array_equal(f, want), np.nonzero(f != want)


SRC2 = """
kernel k(global int A[16]) {
  int v, i;
  for i in 0..4 {
    A[tid] := i;
    barrier;
    v := A[(tid + 1) mod 16];
  }
  v := A[tid * 2 % 16];
}
"""


def test_features_loop_with_barrier():
    p = O.Program(SRC2)
    f = p.features(1, 16, {"A": ("seeded", -5, 300)}, seed=2)
    # statements: for, store, barrier, load, load (5)
    e = {1: (2, 5), 2: (1, 5), 3: (1, 5), 7: (1, 5), 8: (2, 5), 10: (1, 5), 12: sq(5, 256), 13: (1, 8),
         # every pair with the store inside the barrier loop is counted apart
         23: sq(3, 8), 25: sq(1, 16), 27: sq(1, 4), 29: sq(2, 16), 30: sq(1, 8),
         32: 1, 33: 0.5, 34: 0, 35: (1, 8),
         36: -1, 37: 0.5, 38: (1, 16), 39: (2, 8),
         40: -1, 41: (2, 3), 42: 0, 43: (2, 8),
         96: sq(1, 8), 97: sq(1, 8), 98: sq(2, 64), 99: sq(4, 64), 100: sq(3, 64), 101: sq(1, 64),
         102: sq(1, 8)}
    shape = {104: (16, 1024), 105: (1, 1024), 106: (4, 32), 109: (16, 2**20)}
    want = _expect(e, shape)
    avals = [O.seeded_value(2, 0, c, -5, 300) for c in range(16)]
    want[112:120] = _hist(avals, -5, 300, 16).astype(np.float32)
    assert np.array_equal(f, want), np.nonzero(f != want)


SRC3 = """
kernel k(global int A[16], int s) {
  local int L[32];
  int v;
  A[lid] := 1;
  L[v] := 2;
  L[(-3 * tid - 5) mod 32] := v;
  v := L[(tid * 65536 * 65536) mod 32];
  assume(v >= 0);
  assert(v < 100);
  A[(tid * 3) % v] := s;
}
"""


def test_features_not_affine_and_local_arrays():
    p = O.Program(SRC3)
    f = p.features(2, 8, {"A": ("seeded", 0, 16)}, seed=0)
    # statements: store, store, store, load, assume, assert, store (7)
    n = 7
    e = {1: (1, n), 2: (4, n), 4: (1, n), 5: (1, n),
         9: (1, n), 10: (2, n), 11: (2, n), 12: sq(7, 256), 13: (1, 8), 14: (1, 8), 15: (1, 16),
         # self pairs not affine: A[lid], L[v], A[(tid*3) % v]; L pairs with one
         # side not affine: (L[v], L[-3tid-5]), (L[v], L[load]),
         # (L[-3tid-5], L[load]); A pairs: (A[lid], A[% v])
         18: sq(3, 8), 22: sq(4, 8),
         24: 0, 25: sq(2, 16), 30: sq(1, 8),
         32: 1, 33: -2, 34: -2, 35: (1, 8),
         36: 1, 37: -2, 38: -2, 39: (1, 8),
         40: 1, 41: -0.75, 42: (27, 32), 43: (1, 8),
         44: -1, 45: -2, 46: -2, 47: (1, 8),
         48: 1, 49: -2, 50: -2, 51: (1, 8),
         98: sq(5, 64), 100: sq(5, 64), 101: sq(4, 64), 102: sq(2, 8)}
    shape = {104: (8, 1024), 105: (2, 1024), 106: (4, 32), 108: (32, 65536), 109: (16, 2**20)}
    want = _expect(e, shape)
    avals = [O.seeded_value(0, 0, c, 0, 16) for c in range(16)]
    want[112:120] = _hist(avals, 0, 16, 16).astype(np.float32)
    assert np.array_equal(f, want), np.nonzero(f != want)


def test_features_depend_on_seed_only_in_the_histograms():
    p = O.Program(SRC1)
    a = p.features(3, 40, {"A": ("seeded", 0, 16), "B": ("seeded", 0, 1 << 32)}, seed=1)
    b = p.features(3, 40, {"A": ("seeded", 0, 16), "B": ("seeded", 0, 1 << 32)}, seed=2)
    assert np.array_equal(a[:112], b[:112])
    assert not np.array_equal(a[112:], b[112:])
    assert abs(a[112:120].sum() - 64 / 256) < 1e-7 and abs(a[120:128].sum() - 8 / 256) < 1e-7


def test_features_full_width_seeded_range():
    # [0, 2^32) wraps into negative int32 values; the bin is the draw's offset
    # (v - lo) mod 2^32 in eighths of the range
    p = O.Program(SRC1)
    for lo in (0, -2**31, -7):
        f = p.features(1, 64, {"A": ("seeded", lo, lo + 2**32), "B": ("seeded", 0, 16)}, seed=9)
        want = np.zeros(8)
        for c in range(64):
            u = (O.seeded_value(9, 0, c, lo, lo + 2**32) - lo) % 2**32
            want[u * 8 // 2**32] += 1
        assert np.array_equal(f[112:120], (want / 256).astype(np.float32))


SRC_MEET = """
kernel k(global int A[64], global int B[4096]) {
  int v;
  A[(tid * 4) mod 64] := tid;
  v := A[(tid * 4 + 2) mod 64];
  v := A[(tid * 4 + 8) mod 64];
  v := A[(tid * 4 - 8) mod 64];
  B[(tid * 3 + 5) mod 4096] := v;
  v := B[(tid * 3 + 3080) mod 4096];
  v := B[(tid * 3 + 2) mod 4096];
}
"""


def test_features_shifted_pairs_that_meet():
    """Pairs with equal a and different b (feature 19) and those of them
    whose cells meet within 1024 work-items (feature 31), worked by hand:
    A: store at 4t, loads at 4t+2 (4d = 2 mod 64 has no solution), 4t+8
    (d = 2) and 4t-8 (d = -2); B: store at 3t+5, loads at 3t+3080 (3d =
    3075 mod 4096 only for d = 1025 mod 4096) and 3t+2 (d = -1)."""
    f = O.Program(SRC_MEET).features(1, 64, {"A": ("seeded", 0, 16), "B": ("seeded", 0, 16)}, seed=3)
    assert f[19] == np.float32(5) / np.float32(13)
    assert f[31] == np.float32(3) / np.float32(11)
