"""Pins of the workload simulators of the oracle against independent
references: closed forms per object, textbook cellular automata by a library
convolution, a second brute-force agent simulation on tiny grids, and
closed-form / double-precision n-body values."""
import numpy as np
import pytest
from scipy.signal import convolve2d

from oracle import core
from paper_1810_11765_amd import inputs

# ------------------------------------------------------------ alloc microbench


def _c1_closed_form(seed, n, rounds):
    """Per lineage (low 18 id bits), vectorized over all lineages at once."""
    ids = np.arange(n, dtype=np.uint64)
    x = inputs.u01(inputs.ctr(seed, 0, ids, 0))
    v = inputs.u01(inputs.ctr(seed, 0, ids, 1))
    out = []
    for r in range(rounds):
        v = (v + np.float32(0.5) * x).astype(np.float32)
        h = inputs.splitmix64(np.uint64(seed) ^ ids ^ np.uint64(r))
        die = (h & np.uint64(1)).astype(bool)
        nid = (np.uint64(r + 1) << np.uint64(18)) | (ids & np.uint64(0x3FFFF))
        ids = np.where(die, nid, ids)
        x = np.where(die, inputs.u01(inputs.ctr(seed, r + 1, nid, 0)), x)
        v = np.where(die, inputs.u01(inputs.ctr(seed, r + 1, nid, 1)), v)
        o = np.argsort(ids)
        out.append((ids[o].astype(np.int32), x[o], v[o]))
    return out


@pytest.mark.parametrize("seed", [42, 7])
def test_c1_matches_per_lineage_closed_form(seed):
    n = 4096 * 4
    ids, x, v = inputs.alloc_bench_initial(seed, 4096, 4)
    got = core.c1_run(seed, ids, x, v, 10)
    want = _c1_closed_form(seed, n, 10)
    for (gi, gx, gv), (wi, wx, wv) in zip(got, want):
        assert np.array_equal(gi, wi)
        assert np.array_equal(gx.view(np.uint32), wx.view(np.uint32))
        assert np.array_equal(gv.view(np.uint32), wv.view(np.uint32))


def test_c1_invariants_full_size():
    seed = 42
    ids, x, v = inputs.alloc_bench_initial(seed, 65536, 4)
    states = core.c1_run(seed, ids, x, v, 10)
    prev = set(range(262144))
    for r, (i, xx, vv) in enumerate(states):
        assert len(i) == 262144 and len(np.unique(i)) == 262144
        low = np.sort(i & 0x3FFFF)
        assert np.array_equal(low, np.arange(262144))            # one object per lineage
        changed = len(set(i.tolist()) - prev)
        assert abs(changed - 131072) < 5 * 256                   # Binomial(262144, 1/2)
        prev = set(i.tolist())
        assert (xx >= 0).all() and (xx < 1).all()

# ----------------------------------------------------------------- Life-like


def _life_scipy(alive, W, H, steps):
    g = alive.reshape(H, W).astype(np.int32)
    k = np.ones((3, 3), dtype=np.int32); k[1, 1] = 0
    hist = [g.copy()]
    for _ in range(steps):
        nb = convolve2d(g, k, mode="same", boundary="wrap")
        g = ((nb == 3) | ((g == 1) & (nb == 2))).astype(np.int32)
        hist.append(g.copy())
    return hist


def test_life_matches_library_convolution_and_ages():
    W, H, steps = 64, 48, 60
    a0 = inputs.life_initial(3, W, H)
    alive, age = core.c2_run(a0, W, H, steps)
    hist = _life_scipy(a0, W, H, steps)
    assert np.array_equal(alive.reshape(H, W), hist[-1])
    # agent age = number of steps the cell has been alive without interruption
    run = np.zeros((H, W), dtype=np.int32)
    for t in range(1, steps + 1):
        run = np.where((hist[t] == 1) & (hist[t - 1] == 1), run + 1, 0)
    want = np.where(hist[-1] == 1, run, -1)
    assert np.array_equal(age.reshape(H, W), want)


def _grid(W, H, cells):
    a = np.zeros(W * H, dtype=np.uint8)
    for x, y in cells:
        a[y * W + x] = 1
    return a


def test_life_textbook_patterns():
    W = H = 16
    blinker = _grid(W, H, [(5, 6), (6, 6), (7, 6)])
    a1, _ = core.c2_run(blinker, W, H, 1)
    assert set(np.nonzero(a1)[0]) == {5 * W + 6, 6 * W + 6, 7 * W + 6}
    a2, age2 = core.c2_run(blinker, W, H, 2)
    assert np.array_equal(a2, blinker)
    assert age2[6 * W + 6] == 2 and age2[6 * W + 5] == 0          # center survives, ends reborn
    block = _grid(W, H, [(2, 2), (3, 2), (2, 3), (3, 3)])
    a, age = core.c2_run(block, W, H, 7)
    assert np.array_equal(a, block) and (age[block == 1] == 7).all()
    glider = _grid(W, H, [(1, 0), (2, 1), (0, 2), (1, 2), (2, 2)])
    a, _ = core.c2_run(glider, W, H, 4)
    moved = _grid(W, H, [(2, 1), (3, 2), (1, 3), (2, 3), (3, 3)])
    assert np.array_equal(a, moved)
    a, _ = core.c2_run(glider, W, H, 4 * W)                       # full lap on the torus
    assert np.array_equal(a, glider)

# --------------------------------------------------------------- predator-prey


def _wator_bruteforce(kind0, W, H, seed, steps, fb=3, sb=8, gain=4, e0=4):
    """Agent-list simulation: separate objects, explicit phase snapshots."""
    agents = []   # dicts: kind, pos, age, energy
    for c in range(W * H):
        if kind0[c]:
            agents.append(dict(kind=int(kind0[c]), pos=c, age=0, energy=e0 if kind0[c] == 2 else 0))

    def nbrs(c):
        x, y = c % W, c // W
        return [((y - 1) % H) * W + x, y * W + (x + 1) % W, ((y + 1) % H) * W + x, y * W + (x - 1) % W]

    def occ():
        return {a["pos"]: a for a in agents}

    for s in range(1, steps + 1):
        for kind, stream in ((1, 1), (2, 2)):
            o = occ()
            movers = [a for a in agents if a["kind"] == kind]
            claims = {}
            for a in movers:
                a["age"] += 1
                nb = nbrs(a["pos"])
                cand = [c for c in nb if c in o and o[c]["kind"] == 1] if kind == 2 else []
                if not cand:
                    cand = [c for c in nb if c not in o]
                a["want"] = None
                if cand:
                    h = core.ctr(seed, s, a["pos"], stream)
                    t = cand[(h >> 32) % len(cand)]
                    a["want"] = t
                    claims[t] = min(claims.get(t, 1 << 40), a["pos"])
            born, dead = [], []
            for a in movers:
                t = a["want"]
                if t is not None and claims[t] == a["pos"]:
                    if kind == 2:
                        prey = [b for b in agents if b["pos"] == t and b["kind"] == 1 and b not in dead]
                        if prey:
                            dead.append(prey[0]); a["energy"] += gain
                    old = a["pos"]; a["pos"] = t
                    if a["age"] >= (fb if kind == 1 else sb):
                        a["age"] = 0
                        born.append(dict(kind=kind, pos=old, age=0, energy=e0 if kind == 2 else 0))
                if kind == 2:
                    a["energy"] -= 1
                    if a["energy"] <= 0:
                        dead.append(a)
            agents = [a for a in agents if not any(a is d for d in dead)] + born
    kind = np.zeros(W * H, dtype=np.uint8); age = np.zeros(W * H, dtype=np.int32)
    en = np.zeros(W * H, dtype=np.int32)
    for a in agents:
        assert kind[a["pos"]] == 0, "two agents on one cell"
        kind[a["pos"]] = a["kind"]; age[a["pos"]] = a["age"]; en[a["pos"]] = a["energy"]
    return kind, age, en


@pytest.mark.parametrize("seed,W,H", [(1, 7, 5), (2, 9, 9), (42, 12, 10), (7, 16, 3)])
def test_wator_matches_agent_list_bruteforce(seed, W, H):
    k0 = inputs.wator_initial(seed, W, H, fish=0.35, shark=0.15)
    steps = 30
    ok, oa, oe = core.c3_run(k0, W, H, seed, steps)
    bk, ba, be = _wator_bruteforce(k0, W, H, seed, steps)
    assert np.array_equal(ok, bk)
    assert np.array_equal(oa[ok > 0], ba[bk > 0])
    assert np.array_equal(oe[ok == 2], be[bk == 2])


def test_wator_hand_cases():
    W = H = 5
    k0 = np.zeros(25, dtype=np.uint8); k0[12] = 2                   # lone shark
    for steps, alive in ((3, 1), (4, 0)):
        k, _, e = core.c3_run(k0, W, H, 9, steps)
        assert (k == 2).sum() == alive
        if alive:
            assert e[k == 2][0] == 4 - steps                          # one energy per step
    k0 = np.zeros(25, dtype=np.uint8); k0[12] = 1                   # lone fish
    k, a, _ = core.c3_run(k0, W, H, 9, 2)
    assert (k == 1).sum() == 1 and a[k == 1][0] == 2 and k[12] == 0   # moved, aged
    k, a, _ = core.c3_run(k0, W, H, 9, 3)
    assert (k == 1).sum() == 2 and sorted(a[k == 1]) == [0, 0]         # bred at age 3
    # shark next to a fish eats it (fish is boxed in by sharks? no: fish moves first)
    k0 = np.full(25, 0, dtype=np.uint8)
    k0[[11, 13, 7, 17]] = 2; k0[12] = 1                              # fish surrounded by sharks
    k, _, e, cnt = core.c3_run(k0, W, H, 9, 1, with_counts=True)
    assert (k == 1).sum() == 0 and cnt[0, 2] == 1                    # eaten
    assert sorted(e[k == 2]) == [3, 3, 3, 7]                          # the eater gained 4


def test_wator_population_accounting_full_size_short():
    k0 = inputs.wator_initial(42, 256, 256)
    k, a, e, cnt = core.c3_run(k0, 256, 256, 42, 40, with_counts=True)
    f0, s0 = int((k0 == 1).sum()), int((k0 == 2).sum())
    for s in range(40):
        nf, ns, eaten, starved, fb, sb = (int(v) for v in cnt[s])
        assert nf == f0 + fb - eaten and ns == s0 + sb - starved
        f0, s0 = nf, ns
    assert (k == 1).sum() == f0 and (k == 2).sum() == s0
    assert (e[k == 2] >= 1).all() and (a[k > 0] >= 0).all()

# -------------------------------------------------------------------- n-body


def test_nbody_two_body_closed_form():
    ids = np.array([0, 1], dtype=np.int32)
    x = np.array([0.0, 0.5], dtype=np.float32); y = np.array([0.0, 0.25], dtype=np.float32)
    z = np.zeros(2, dtype=np.float32); m = np.array([2.0, 3.0], dtype=np.float32)
    (i2, x2, y2, vx2, vy2, m2), npairs = core.c4_step(ids, x, y, z, z, m, G=1e-2, dt=0.1)
    assert npairs == 0 and len(i2) == 2
    d = np.hypot(0.5, 0.25)
    a0 = 1e-2 * 3.0 / d**3 * np.array([0.5, 0.25])
    a1 = -1e-2 * 2.0 / d**3 * np.array([0.5, 0.25])
    np.testing.assert_allclose([vx2[0], vy2[0]], a0 * 0.1, rtol=1e-6)
    np.testing.assert_allclose([vx2[1], vy2[1]], a1 * 0.1, rtol=1e-6)
    np.testing.assert_allclose([x2[0], y2[0]], a0 * 0.01, rtol=1e-6)


def test_nbody_merge_chain_conserves_mass_and_momentum():
    # 0-1 and 1-2 closer than 1e-4, 0-2 farther: one component merging into id 0
    ids = np.array([0, 1, 2, 3], dtype=np.int32)
    x = np.array([0.1, 0.10008, 0.10016, 0.5], dtype=np.float32)
    y = np.array([0.0, 0.0, 0.0, 0.5], dtype=np.float32)
    vx = np.array([1.0, -2.0, 0.5, 0.0], dtype=np.float32)
    vy = np.array([0.0, 1.0, 3.0, 0.0], dtype=np.float32)
    m = np.array([1.0, 2.0, 4.0, 1.0], dtype=np.float32)
    (i2, x2, y2, vx2, vy2, m2), npairs = core.c4_step(ids, x, y, vx, vy, m, G=0.0, dt=0.0)
    assert npairs == 2 and list(i2) == [0, 3]
    assert m2[0] == 7.0 and x2[0] == np.float32(0.1)
    np.testing.assert_allclose(vx2[0], (1 - 4 + 2) / 7, rtol=1e-6)
    np.testing.assert_allclose(vy2[0], (0 + 2 + 12) / 7, rtol=1e-6)


def test_nbody_step_against_double_precision_and_no_close_pairs():
    n = 512
    x, y, vx, vy, m = inputs.nbody_initial(5, n)
    x[1] = x[0] + np.float32(3e-5); y[1] = y[0]                     # force one merge
    ids = np.arange(n, dtype=np.int32)
    (i2, x2, y2, vx2, vy2, m2), npairs = core.c4_step(ids, x, y, vx, vy, m)
    assert npairs >= 1 and 1 not in set(i2.tolist())
    assert abs(float(m2.sum(dtype=np.float64)) - float(m.sum(dtype=np.float64))) < 1e-4
    # double-precision acceleration of the survivors (positions unchanged by merging)
    # survivors keep their positions through the merge phase, so the force
    # phase sees the initial positions of the surviving ids
    X0, Y0, Mm = x[i2].astype(np.float64), y[i2].astype(np.float64), m2.astype(np.float64)
    dx = X0[None, :] - X0[:, None]; dy = Y0[None, :] - Y0[:, None]
    d2 = dx * dx + dy * dy; np.fill_diagonal(d2, 1.0)
    s = 1e-6 * Mm[None, :] / (d2 * np.sqrt(d2)); np.fill_diagonal(s, 0.0)
    ax = (s * dx).sum(1); ay = (s * dy).sum(1)
    surv0 = i2[i2 != 0]                                               # untouched by the merge
    sel = np.searchsorted(i2, surv0)
    np.testing.assert_allclose(vx2[sel], vx[surv0] + ax[sel] * 1e-3, rtol=2e-4, atol=1e-9)
    np.testing.assert_allclose(vy2[sel], vy[surv0] + ay[sel] * 1e-3, rtol=2e-4, atol=1e-9)
    # after the merge phase no two survivors are closer than the threshold
    d = np.sqrt(d2 + np.eye(len(X0)))
    assert d.min() >= 1e-4 * 0.999


def _inject_close_pairs(x, y, rng, k, chain=False):
    """Put k bodies within 3e-5 of another body (and some 3-chains)."""
    n = len(x)
    for _ in range(k):
        i, j = rng.choice(n, 2, replace=False)
        x[j] = x[i] + np.float32(3e-5) * np.float32(rng.uniform(-1, 1))
        y[j] = y[i] + np.float32(3e-5) * np.float32(rng.uniform(-1, 1))
        if chain:
            l = rng.choice(n)
            x[l] = x[j] + np.float32(6e-5); y[l] = y[j]


def test_grid_merge_equals_bruteforce_merge():
    rng = np.random.default_rng(0)
    n = 3000
    x, y, vx, vy, m = inputs.nbody_initial(9, n)
    vx = rng.standard_normal(n).astype(np.float32); vy = rng.standard_normal(n).astype(np.float32)
    _inject_close_pairs(x, y, rng, 40, chain=True)
    ids = np.arange(n, dtype=np.int32)
    brute, nb = core.c4_step(ids, x, y, vx, vy, m, G=0.0, dt=0.0)      # G = dt = 0: merge only
    grid, ng = core.c4_merge_grid(ids, x, y, vx, vy, m)
    assert nb == ng and nb >= 40
    for a, b in zip(brute, grid):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_c4_accel_equals_the_force_phase_of_a_step_bit_for_bit():
    """c4_accel (used to check large states body by body) is the force phase
    of c4_step: with bodies at rest, dt = 1 and no close pairs, a step sets
    v = 0 + a*1 = a exactly, so the step's velocities are the accelerations."""
    n = 700
    x, y, vx, vy, m = inputs.nbody_initial(11, n)
    ids = np.arange(n, dtype=np.int32)
    (i2, _, _, vx2, vy2, _), npairs = core.c4_step(ids, x, y, vx, vy, m, G=1e-6, dt=1.0)
    assert npairs == 0 and len(i2) == n
    ax, ay = core.c4_accel(x, y, m, np.arange(n), G=1e-6)
    assert np.array_equal(ax.view(np.uint32), vx2.view(np.uint32))
    assert np.array_equal(ay.view(np.uint32), vy2.view(np.uint32))
    # a subset gives the same values as the full selection
    sel = np.array([0, 5, n - 1, 321], dtype=np.int64)
    sx, sy = core.c4_accel(x, y, m, sel, G=1e-6)
    assert np.array_equal(sx.view(np.uint32), ax[sel].view(np.uint32))
    assert np.array_equal(sy.view(np.uint32), ay[sel].view(np.uint32))


@pytest.mark.parametrize("n,seed", [(2, 3), (64, 4), (512, 5)])
def test_c4_accel_against_double_precision(n, seed):
    """The float32 sum in ascending id stays within 2e-4 of the double-precision
    sum, relative to the sum of the terms' magnitudes (n * 2^-24 bounds the
    summation error, a few ulps the terms themselves)."""
    x, y, _, _, m = inputs.nbody_initial(seed, n)
    ax, ay = core.c4_accel(x, y, m, np.arange(n), G=1e-6)
    X, Y, Mm = x.astype(np.float64), y.astype(np.float64), m.astype(np.float64)
    dx = X[None, :] - X[:, None]
    dy = Y[None, :] - Y[:, None]
    d2 = dx * dx + dy * dy
    np.fill_diagonal(d2, 1.0)
    s = 1e-6 * Mm[None, :] / (d2 * np.sqrt(d2))
    np.fill_diagonal(s, 0.0)
    for got, comp in ((ax, s * dx), (ay, s * dy)):
        want = comp.sum(1)
        scale = np.abs(comp).sum(1)
        assert (np.abs(got - want) <= 2e-4 * scale + 1e-30).all()


def test_grid_step_equals_bruteforce_step():
    """The whole grid-merge step (used for the full-size golden values) equals
    the brute-force step over two steps, merges included."""
    rng = np.random.default_rng(1)
    n = 2500
    x, y, vx, vy, m = inputs.nbody_initial(12, n)
    _inject_close_pairs(x, y, rng, 25, chain=True)
    ids = np.arange(n, dtype=np.int32)
    a, _ = core.c4_step(ids, x, y, vx, vy, m)
    a, _ = core.c4_step(*a)
    b = core.c4_run_grid(ids, x, y, vx, vy, m, 2)
    assert len(a[0]) < n
    for p, q in zip(a, b):
        assert np.array_equal(p.view(np.uint32), q.view(np.uint32))
