"""Pins of the CPU oracle to what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the paper's
printed worked examples and table counts, a textbook Sylvester Hadamard matrix
(Lemma 3 via a differently computed Alg. 2), exhaustive covering on tiny
inputs (Theorem 1 / Corollary 1), a GF(2)-rank closed form for the number of
colliding functions, a statistical check of Theorem 2 property 2, and brute
force on tiny inputs.  None of them needs a GPU.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.linalg import hadamard

import oracle
import synth

P31 = (1 << 31) - 1


def str_point(s):
    """Paper string (coordinates 1..d left to right) -> uint64 words."""
    d = len(s)
    w = np.zeros((d + 63) // 64, np.uint64)
    for k, ch in enumerate(s):
        if ch == "1":
            w[k >> 6] |= np.uint64(1) << np.uint64(k & 63)
    return w


def mask_str(row):
    return "".join("1" if v else "0" for v in row)


def pattern_key(s):
    """Key of a masked pattern when b_c = 2^c and P > 2^d: the pattern read as
    an integer with coordinate c at bit c."""
    return sum(1 << k for k, ch in enumerate(s) if ch == "1")


def pow2_params(d, rpart, cols, P=P31):
    return oracle.explicit_params(d, rpart, np.zeros(d, np.int32), cols,
                                  [1 << c for c in range(d)], P)


# --------------------------------------------------------------------------
# Worked examples
# --------------------------------------------------------------------------

def test_c78_matrix_identity_mapping(golden):
    rows = golden("c78_matrix.txt")
    pr = oracle.explicit_params(8, 2, np.zeros(8, np.int32), np.arange(8), np.ones(8), P31)
    m = oracle.masks(pr)
    assert m.shape == (7, 8)
    assert [mask_str(r) for r in m] == rows


def _example_2_1(golden):
    g = {}
    for ln in golden("example_2_1.txt"):
        k, *v = ln.split()
        g[k] = v
    return g


def test_example_2_1_masks(golden):
    g = _example_2_1(golden)
    d, r = int(g["d"][0]), int(g["r"][0])
    cols = [int(s, 2) for s in g["m"]]
    pr = oracle.explicit_params(d, r, np.zeros(d, np.int32), cols, np.ones(d), P31)
    m = oracle.masks(pr)
    assert [mask_str(row) for row in m] == [g[f"g{v}"][0] for v in range(1, 8)]


def test_example_2_1_single_collision_keys(golden):
    g = _example_2_1(golden)
    d, r = int(g["d"][0]), int(g["r"][0])
    cols = [int(s, 2) for s in g["m"]]
    pr = pow2_params(d, r, cols)
    x, q = str_point(g["x"][0]), str_point(g["q"][0])
    k = oracle.keys(np.stack([x, q]), pr)
    equal = np.nonzero(k[:, 0] == k[:, 1])[0]
    v, val = int(g["collide"][0]), g["collide"][1]
    assert list(equal) == [v - 1]
    assert int(k[v - 1, 0]) == pattern_key(val)


def test_example_3_1_collisions(golden):
    g = {ln.split()[0]: ln.split()[1:] for ln in golden("example_3_1.txt")}
    pr = pow2_params(8, 2, list(range(8)))
    pts = np.stack([str_point(g[k][0]) for k in ("x", "y", "q")])
    k = oracle.keys(pts, pr)
    row, val = int(g["collide_x"][0]), g["collide_x"][1]
    assert list(np.nonzero(k[:, 0] == k[:, 2])[0]) == [row - 1]
    assert int(k[row - 1, 0]) == pattern_key(val)
    assert g["collide_y"] == ["none"]
    assert not np.any(k[:, 1] == k[:, 2])


def test_printed_table_counts(golden):
    for ln in golden("table_counts.txt"):
        r, t, L = map(int, ln.split())
        assert oracle.parts_for_radius(r) == t
        pr = oracle.derive_params(64, r, seed=7)
        assert pr.t == t and pr.L == L


def _bits_to_words(bits: str) -> np.ndarray:
    # coordinates 1..d left to right -> bit c-1 of the packed point
    w = np.zeros((1, (len(bits) + 63) // 64), np.uint64)
    for c, ch in enumerate(bits):
        if ch == "1":
            w[0, c // 64] |= np.uint64(1) << np.uint64(c % 64)
    return w


def test_replication_example(golden):
    for ln in golden("replication.txt"):
        f = ln.split()
        if f[0] != "example":
            continue
        bits, times, want = f[1], int(f[2]), f[3]
        got = oracle.replicate(_bits_to_words(bits), len(bits), times)
        assert np.array_equal(got, _bits_to_words(want))


def test_replication_table_counts(golden):
    # Fig. 3's replication: the family of radius times * r on the replicated
    # points, one part
    for ln in golden("replication.txt"):
        f = ln.split()
        if f[0] != "tables":
            continue
        r, times, L = int(f[1]), int(f[2]), int(f[3])
        pr = oracle.derive_params(times * 128, times * r, seed=7, override_t=1)
        assert pr.t == 1 and pr.L == L


@pytest.mark.parametrize("d,r,times,seed", [(6, 1, 3, 1), (8, 1, 2, 2), (5, 2, 2, 3)])
def test_replication_covering_exhaustive(d, r, times, seed):
    # Theorem 1 on the replicated points: a difference of at most r becomes
    # one of at most times * r, which the family of that radius covers
    pr = oracle.derive_params(times * d, times * r, seed, override_t=1)
    m = oracle.masks(pr).astype(bool)
    for pos in _all_z(d, r):
        z = np.zeros((1, 1), np.uint64)
        for c in pos:
            z[0, 0] |= np.uint64(1) << np.uint64(c)
        zz = oracle.replicate(z, d, times)
        zb = np.array([(int(zz[0, c // 64]) >> (c % 64)) & 1 for c in range(times * d)], bool)
        assert zb.sum() == times * len(pos)
        assert np.any(~np.any(m & zb, axis=1)), f"difference {pos} not covered"


def test_splitmix64_reference_outputs(golden):
    for ln in golden("splitmix64.txt"):
        seed, k, v = ln.split()
        assert oracle.splitmix64(int(seed), int(k)) == int(v, 16)


# --------------------------------------------------------------------------
# Lemma 3: Alg. 2 (fast Hadamard transform) reaches exactly the Eq. (1) keys
# of the basic masks.  Here Alg. 2 is computed independently with a textbook
# Sylvester Hadamard matrix in exact Python integers.
# --------------------------------------------------------------------------

def alg2_keys_textbook(x_bits, pr):
    D = pr.D
    H = hadamard(D).astype(object)
    out = []
    for p in range(pr.t):
        qt = [int(pr.b[c]) if (x_bits[c] and pr.part[c] == p) else 0 for c in range(pr.d)]
        tvec = [0] * D
        for c in range(pr.d):
            tvec[int(pr.col[c])] += qt[c]
        norm1 = sum(qt)
        F = H.dot(np.array(tvec, dtype=object))
        h = [((norm1 - int(F[v])) // 2) % pr.P for v in range(D)]
        assert all((norm1 - int(F[v])) % 2 == 0 for v in range(D))
        assert h[0] == 0  # the all-zero codeword, removed by Alg. 2
        out.extend(h[1:])
    return out


@pytest.mark.parametrize("d,r,t,seed", [
    (12, 2, 0, 1),    # general: d > 2^(r+1)
    (8, 2, 0, 2),     # specific: d == 2^(r+1)
    (5, 2, 0, 3),     # specific with 0-padding
    (40, 10, 0, 4),   # 2 partitions, general per part
    (23, 6, 2, 5),    # 2 partitions of unequal size (remainder to the last)
    (30, 4, 3, 6),    # 3 partitions
    (70, 3, 0, 7),    # multi-word point
])
def test_lemma3_fht_equals_basic_keys(d, r, t, seed):
    pr = oracle.derive_params(d, r, seed, override_t=t)
    rng = np.random.default_rng(seed)
    pts = synth.uniform_points(12, d, rng)
    k = oracle.keys(pts, pr)
    for i in range(pts.shape[0]):
        bits = [int((pts[i, c >> 6] >> np.uint64(c & 63)) & np.uint64(1)) for c in range(d)]
        assert [int(v) for v in k[:, i]] == alg2_keys_textbook(bits, pr)


def test_lemma3_with_small_prime():
    # Lemma 3 holds for any prime and any seed vector b in [P]^d
    d, r = 16, 3
    pr0 = oracle.derive_params(d, r, 11, P=10007)
    assert int(pr0.b.max()) < 10007
    pts = synth.uniform_points(8, d, np.random.default_rng(3))
    k = oracle.keys(pts, pr0)
    for i in range(8):
        bits = [int((pts[i, 0] >> np.uint64(c)) & np.uint64(1)) for c in range(d)]
        assert [int(v) for v in k[:, i]] == alg2_keys_textbook(bits, pr0)


# --------------------------------------------------------------------------
# Covering (Theorem 1, Lemma 2, Corollary 1): every difference pattern z with
# |z| <= r is missed by at least one mask, for every mapping.
# --------------------------------------------------------------------------

def _all_z(d, r):
    for k in range(r + 1):
        for pos in itertools.combinations(range(d), k):
            yield pos


@pytest.mark.parametrize("d,r,t,seed", [(8, 2, 0, 1), (10, 2, 0, 2), (6, 1, 0, 3),
                                        (12, 3, 0, 4), (16, 4, 2, 5), (14, 5, 2, 6)])
def test_covering_exhaustive(d, r, t, seed):
    pr = oracle.derive_params(d, r, seed, override_t=t)
    m = oracle.masks(pr).astype(bool)
    for pos in _all_z(d, r):
        z = np.zeros(d, bool)
        z[list(pos)] = True
        assert np.any(~np.any(m & z, axis=1)), f"difference {pos} not covered"


@pytest.mark.parametrize("cols", [[0] * 10, [5] * 10, [1, 2, 3, 4, 5, 6, 7, 1, 2, 3]])
def test_covering_any_mapping(cols):
    # Theorem 1 holds for *every* mapping, including degenerate ones
    d, r = 10, 2
    pr = oracle.explicit_params(d, r, np.zeros(d, np.int32), cols, np.ones(d), P31)
    m = oracle.masks(pr).astype(bool)
    for pos in _all_z(d, r):
        z = np.zeros(d, bool)
        z[list(pos)] = True
        assert np.any(~np.any(m & z, axis=1))


def test_covering_through_keys():
    # Theorem 2 property 1 at the key level: equal masked values give equal keys
    d, r = 64, 6
    pr = oracle.derive_params(d, r, 99)
    rng = np.random.default_rng(5)
    x = synth.uniform_points(1, d, rng)[0]
    ys = np.stack([synth.flip_distinct(x, d, int(rng.integers(0, r + 1)), rng) for _ in range(200)])
    k = oracle.keys(np.vstack([x[None], ys]), pr)
    assert np.all(np.any(k[:, 1:] == k[:, :1], axis=0))


# --------------------------------------------------------------------------
# Closed form for the number of colliding functions: within part p the mask
# of v misses the difference set Z_p iff v is orthogonal (over GF(2)) to every
# column m(c), c in Z_p, so exactly 2^(r'+1-rank_p) - 1 non-zero v collide.
# --------------------------------------------------------------------------

def gf2_rank(vectors):
    basis = []
    for v in vectors:
        for b in basis:
            v = min(v, v ^ b)
        if v:
            basis.append(v)
    return len(basis)


@pytest.mark.parametrize("d,r,t,seed", [(64, 6, 0, 1), (40, 10, 0, 2), (20, 3, 0, 3), (90, 8, 3, 4)])
def test_collision_count_closed_form(d, r, t, seed):
    pr = oracle.derive_params(d, r, seed, override_t=t)
    m = oracle.masks(pr).astype(bool)
    rng = np.random.default_rng(seed)
    for _ in range(60):
        k = int(rng.integers(0, 2 * r + 2))
        z = np.zeros(d, bool)
        z[rng.choice(d, size=k, replace=False)] = True
        got = int(np.sum(~np.any(m & z, axis=1)))
        want = 0
        for p in range(pr.t):
            cols = [int(pr.col[c]) for c in range(d) if z[c] and pr.part[c] == p]
            want += 2 ** (pr.rpart + 1 - gf2_rank(cols)) - 1
        assert got == want


def test_theorem2_property2_statistical():
    # E[#colliding functions] < 2^(r+1-dist) over random mappings / permutations
    rng = np.random.default_rng(17)
    for d, r in [(16, 3), (40, 3)]:  # specific (d <= 2^(r+1)) and general
        for dist in range(1, 7):
            tot = 0
            trials = 400
            for s in range(trials):
                pr = oracle.derive_params(d, r, 1000 * dist + s)
                z = rng.choice(d, size=dist, replace=False)
                cols = [int(pr.col[c]) for c in z]
                tot += 2 ** (r + 1 - gf2_rank(cols)) - 1
            mean = tot / trials
            assert mean < 2 ** (r + 1 - dist) * 1.05 + 0.05, (d, r, dist, mean)


# --------------------------------------------------------------------------
# Alg. 1: which pre-processing branch, and how many copies or parts
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 1000, 65536, 1 << 20, 10 ** 7, 1 << 40])
@pytest.mark.parametrize("c", [1.1, 1.5, 2.0, 3.0])
def test_preprocessing_keeps_tables_near_n_to_1_over_c(n, c):
    # The pre-processing exists to keep the radius the family is drawn for
    # at about log(n)/c, so that a part has about n^(1/c) tables: the chosen
    # copies (or parts) leave that radius at most log(n)/c, and one copy
    # more (or one part fewer) would push it over.
    logn = math.log2(n)
    for r in range(1, 41):
        k, t = oracle.preprocessing(n, r, c)
        assert k >= 1 and t >= 1 and (k == 1 or t == 1)
        if c * r < logn:
            assert t == 1 and c * k * r <= logn < c * (k + 1) * r
            assert 2 ** (k * r + 1) - 1 < 2 * n ** (1 / c)
        elif c * r > logn:
            assert k == 1 and c * r / t <= logn
            assert t == 1 or c * r / (t - 1) > logn
            assert 2 ** (r // t + 1) - 1 < 2 * n ** (1 / c)
        else:
            assert (k, t) == (1, 1)


def test_preprocessing_special_cases():
    # c r = log n takes neither branch; small radii replicate, large ones split
    assert oracle.preprocessing(65536, 8, 2.0) == (1, 1)
    assert oracle.preprocessing(65536, 2, 2.0) == (4, 1)
    assert oracle.preprocessing(65536, 1, 1.5) == (10, 1)
    assert oracle.preprocessing(1 << 20, 20, 2.0) == (1, 2)
    assert oracle.preprocessing(1 << 20, 21, 2.0) == (1, 3)


# --------------------------------------------------------------------------
# Sec. 3.3 variant: the coordinate map never targets column 0
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,r,t,seed", [(6, 2, 0, 1), (7, 2, 0, 2), (8, 2, 0, 3), (12, 2, 0, 4),
                                        (16, 4, 0, 5), (14, 5, 2, 6)])
def test_exclude_column0_covering_exhaustive(d, r, t, seed):
    # the variant is still r-covering (every difference pattern of weight <= r
    # avoids the mask of some row); its columns are 1..D-1, injective in a
    # part of at most D - 1 coordinates (d = 7 at D = 8 is that boundary,
    # d = 8 already takes the i.i.d. map)
    pr = oracle.derive_params(d, r, seed, override_t=t, exclude_column0=True)
    assert np.all((pr.col >= 1) & (pr.col < pr.D))
    for q in range(pr.t):
        cq = pr.col[pr.part == q]
        if len(cq) <= pr.D - 1:
            assert len(set(cq.tolist())) == len(cq)
    m = oracle.masks(pr).astype(bool)
    for pos in _all_z(d, r):
        z = np.zeros(d, bool)
        z[list(pos)] = True
        assert np.any(~np.any(m & z, axis=1)), f"difference {pos} not covered"


def test_exclude_column0_expected_collisions():
    # General construction (i.i.d. columns): row v != 0 collides on a
    # difference of k coordinates iff all k columns are orthogonal to v.  Of
    # the D - 1 columns other than 0, D/2 - 1 are, so the expected number of
    # colliding rows is (D-1) ((D/2-1)/(D-1))^k, below the bound 2^(r+1-k) of
    # Sec. 3.3 and below (D-1)/2^k, the value when column 0 may be drawn.
    rng = np.random.default_rng(23)
    d, r = 24, 2
    D = 2 ** (r + 1)
    for k in range(1, 5):
        trials = 3000
        vals = np.empty(trials)
        for s in range(trials):
            pr = oracle.derive_params(d, r, 50000 * k + s, exclude_column0=True)
            z = rng.choice(d, size=k, replace=False)
            vals[s] = 2 ** (r + 1 - gf2_rank([int(pr.col[c]) for c in z])) - 1
        exact = (D - 1) * ((D / 2 - 1) / (D - 1)) ** k
        assert abs(vals.mean() - exact) < 0.08, (k, vals.mean(), exact)
        assert exact < 2 ** (r + 1 - k) and exact < (D - 1) / 2 ** k
        if k == 1:
            assert np.all(vals == D / 2 - 1)  # no column is orthogonal to every row


# --------------------------------------------------------------------------
# Parameter draws: structural invariants of Alg. 1 / Alg. 2
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,r,t", [(128, 4, 0), (256, 8, 0), (64, 6, 0), (512, 12, 0),
                                   (256, 10, 0), (1024, 20, 0), (101, 12, 3),
                                   (128, 6, 0), (16, 3, 0), (256, 12, 0)])  # last 3: d' == D
def test_param_invariants(d, r, t):
    pr = oracle.derive_params(d, r, 42, override_t=t)
    tt = t if t else (1 if r < 10 else 2)
    assert pr.t == tt and pr.rpart == r // tt
    sizes = np.bincount(pr.part, minlength=pr.t)
    blk = d // tt
    assert list(sizes[:-1]) == [blk] * (tt - 1) and sizes[-1] == d - blk * (tt - 1)
    assert np.all((pr.col >= 0) & (pr.col < pr.D))
    assert np.all(pr.b < np.uint64(P31))
    for p in range(pr.t):
        cols = pr.col[pr.part == p]
        if cols.size <= pr.D:  # specific construction: a permutation, so injective
            assert np.unique(cols).size == cols.size
    # deterministic in the seed, different across seeds
    pr2 = oracle.derive_params(d, r, 42, override_t=t)
    pr3 = oracle.derive_params(d, r, 43, override_t=t)
    assert np.array_equal(pr.col, pr2.col) and np.array_equal(pr.b, pr2.b)
    assert not np.array_equal(pr.b, pr3.b)
    if tt == 1:
        assert np.all(pr.part == 0)


def test_bounded_draws_uniform():
    # b is uniform over [0, P): a chi-square check on the top 4 bits
    pr = oracle.derive_params(4096, 4, 5)
    hist = np.bincount((pr.b >> np.uint64(27)).astype(np.int64), minlength=16)
    exp = 4096 / 16
    chi2 = float(np.sum((hist - exp) ** 2 / exp))
    assert chi2 < 40  # 15 dof, p ~ 5e-4


# --------------------------------------------------------------------------
# Tables, queries and brute force
# --------------------------------------------------------------------------

def test_tables_sorted_and_complete():
    w = synth.small(0.05)
    pr = oracle.derive_params(w.d, w.r, 3001)
    k = oracle.keys(w.points, pr)
    tk, ti = oracle.tables(k)
    for T in range(pr.L):
        order = np.lexsort((ti[T], tk[T]))
        assert np.array_equal(order, np.arange(w.n))
        assert np.array_equal(np.sort(ti[T]), np.arange(w.n))
        assert np.array_equal(k[T][ti[T]], tk[T])


def test_brute_force_tiny():
    rng = np.random.default_rng(8)
    for d in (5, 64, 70, 130):
        pts = synth.uniform_points(40, d, rng)
        qs = synth.uniform_points(5, d, rng)
        res = oracle.brute_force(pts, d, qs, rq=d // 2)
        for i in range(5):
            qi = sum(int(qs[i, w]) << (64 * w) for w in range(qs.shape[1]))
            want = [j for j in range(40)
                    if bin(qi ^ sum(int(pts[j, w]) << (64 * w) for w in range(pts.shape[1]))).count("1") <= d // 2]
            assert list(res.ids[i]) == want


def test_brute_force_ignores_pad_bits():
    pts = np.array([[0xF0]], np.uint64)  # bits 4..7 set: beyond d = 4
    q = np.array([[0x00]], np.uint64)
    assert list(oracle.brute_force(pts, 4, q, 0).ids[0]) == [0]


@pytest.mark.parametrize("make,seed", [(lambda: synth.small(0.1), 3001),
                                       (lambda: synth.mid(0.004), 3002),
                                       (lambda: synth.learned_code(0.0005), 3003),
                                       (lambda: synth.mixture(4000, 512, 12, 8, 0.01, 50, seed=77), 3004)])
def test_strategy2_total_recall(make, seed):
    w = make()
    pr = oracle.derive_params(w.d, w.r, seed)
    mask = oracle.masks(pr)
    k = oracle.keys(w.points, pr, mask=mask)
    tk, ti = oracle.tables(k)
    qk = oracle.keys(w.queries, pr, mask=mask)
    res = oracle.query_batch(w.points, w.d, tk, ti, w.queries, qk, w.r)
    bf = oracle.brute_force(w.points, w.d, w.queries, w.r)
    assert sum(len(x) for x in bf.ids) > 0
    for i in range(w.nq):
        assert np.array_equal(res.ids[i], bf.ids[i])
        # counters: #Collisions is the summed bucket sizes, #Candidates the
        # number of distinct colliding points
        seen = set()
        coll = 0
        for T in range(pr.L):
            ids = np.nonzero(k[T] == qk[T, i])[0]
            coll += ids.size
            seen.update(ids.tolist())
        assert res.collisions[i] == coll and res.candidates[i] == len(seen)


def test_query_smaller_radius_is_exact():
    # covering for radius r covers every smaller radius
    w = synth.small(0.1)
    pr = oracle.derive_params(w.d, w.r, 3001)
    mask = oracle.masks(pr)
    k = oracle.keys(w.points, pr, mask=mask)
    tk, ti = oracle.tables(k)
    qk = oracle.keys(w.queries, pr, mask=mask)
    for rq in range(w.r + 1):
        res = oracle.query_batch(w.points, w.d, tk, ti, w.queries, qk, rq)
        bf = oracle.brute_force(w.points, w.d, w.queries, rq)
        for i in range(w.nq):
            assert np.array_equal(res.ids[i], bf.ids[i])


# --------------------------------------------------------------------------
# Points given by their nonzero coordinates (Sec. 3.2's sparse setting): the
# sparse keys and linear scan reduce to the dense ones on the same points,
# which are pinned above.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,r,t,seed", [(700, 9, 0, 21), (3000, 29, 3, 22), (257, 4, 0, 23), (1500, 13, 2, 24)])
def test_sparse_keys_equal_dense_keys(d, r, t, seed):
    rng = np.random.default_rng(seed)
    ptr, cols = synth.sparse_rows(40, d, 25.0, 1.0, 0.9, rng)
    ptr = np.concatenate([ptr, [ptr[-1]]])  # and an empty row
    pr = oracle.derive_params(d, r, seed, override_t=t)
    dense = synth.csr_to_words(ptr, cols, d)
    assert np.array_equal(oracle.keys_sparse(ptr, cols, pr), oracle.keys(dense, pr))


def test_sparse_keys_closed_forms():
    # one set coordinate c: key b_c in the tables of its part whose codeword
    # has a one in its column, 0 elsewhere; no coordinate: all keys 0
    d, r = 200, 11
    pr = oracle.derive_params(d, r, 31, override_t=2)
    ptr = np.array([0, 1, 1], np.int64)
    for c in (0, 57, 199):
        k = oracle.keys_sparse(ptr, np.array([c], np.int32), pr)
        for p in range(pr.t):
            for v in range(1, pr.D):
                T = p * pr.Lp + v - 1
                on = p == pr.part[c] and bin(v & int(pr.col[c])).count("1") % 2 == 1
                assert int(k[T, 0]) == (int(pr.b[c]) if on else 0)
        assert not k[:, 1].any()


def test_sparse_brute_force_equal_dense():
    rng = np.random.default_rng(25)
    d = 5000
    ptr, cols = synth.sparse_rows(300, d, 12.0, 1.2, 1.1, rng)
    qptr, qcols = synth.sparse_rows(10, d, 12.0, 1.2, 1.1, rng)
    for rq in (0, 3, 12, 40):
        want = oracle.brute_force(synth.csr_to_words(ptr, cols, d), d, synth.csr_to_words(qptr, qcols, d), rq)
        got = oracle.brute_force_sparse(ptr, cols, qptr, qcols, d, rq)
        assert np.array_equal(got.counts, want.counts)
        for a, b in zip(got.ids, want.ids):
            assert np.array_equal(a, b)


def test_sparse_brute_force_tiny_sets():
    # distance = size of the symmetric difference of the coordinate sets
    ptr = np.array([0, 2, 5, 5], np.int64)
    cols = np.array([1, 9, 1, 2, 9], np.int32)
    qptr = np.array([0, 1], np.int64)
    res = oracle.brute_force_sparse(ptr, cols, qptr, np.array([9], np.int32), 10, 1)
    assert list(res.ids[0]) == [0, 2]  # {1,9}: 1 away, {1,2,9}: 2, {}: 1
