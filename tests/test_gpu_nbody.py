"""GPU parity of the n-body-with-merging workload (device_do all-pairs force,
merge by connected components, destruction) against the CPU oracle.  FP32 is
formed in the same order with one IEEE rounding per operation on both sides
(-ffp-contract=off, correctly rounded / and sqrtf), so the comparison is
bit-exact; the stated tolerance (relative 1e-5) is the fallback bar."""
import numpy as np
import pytest

from helpers import check_heap, say
from oracle import core
from paper_1810_11765_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1810_11765_amd import smmo  # noqa: F401


def W():
    from paper_1810_11765_amd import workloads
    return workloads


def _inject(x, y, rng, k):
    n = len(x)
    for _ in range(k):
        i, j = rng.choice(n, 2, replace=False)
        x[j] = x[i] + np.float32(3e-5) * np.float32(rng.uniform(-1, 1))
        y[j] = y[i] + np.float32(3e-5) * np.float32(rng.uniform(-1, 1))
        if rng.random() < 0.3:                       # chain of three
            l = rng.choice(n)
            x[l] = x[j] + np.float32(7e-5); y[l] = y[j]


def _same(gpu, ora, what):
    for name, a, b in zip(("id", "x", "y", "vx", "vy", "m"), gpu, ora):
        assert a.shape == b.shape, f"{what}: {name} count {a.shape} vs {b.shape}"
        if name == "id":
            assert np.array_equal(a, b), f"{what}: survivor ids differ"
        else:
            if not np.array_equal(a.view(np.uint32), b.view(np.uint32)):
                rel = np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30))
                assert rel <= 1e-5, f"{what}: {name} rel err {rel}"


@pytest.mark.parametrize("n,steps,seed", [(2048, 40, 1), (1000, 30, 2), (64 * 37 + 5, 10, 3)])
def test_nbody_parity_small(n, steps, seed):
    say("nbody small", n, steps)
    rng = np.random.default_rng(seed)
    x, y, vx, vy, m = inputs.nbody_initial(seed, n)
    _inject(x, y, rng, 25)
    sim = W().NBody(n=n, init=(x, y, vx, vy, m), G=1e-4)
    sim.populate()
    ora = (np.arange(n, dtype=np.int32), x, y, vx, vy, m)
    total_pairs = 0
    for s in range(steps):
        sim.step()
        ora, npairs = core.c4_step(*ora, G=1e-4)
        total_pairs += npairs
        if s in (0, steps - 1):
            _same(sim.state(), ora, f"step {s + 1}")
    assert total_pairs >= 25
    check_heap(sim.heap, expect_live=[len(ora[0])])


def test_nbody_full_size_sampled():
    """262,144 bodies, one step: the merge phase against the oracle on the
    whole state, the all-pairs force (device_do over 4,096 blocks) on sampled
    bodies."""
    say("nbody full")
    n = 262144
    sim = W().NBody(n=n)
    sim.populate()
    state = (np.arange(n, dtype=np.int32),) + sim.init
    sim.merge()
    merged, npairs = core.c4_merge_grid(*state)
    _same(sim.state(), merged, "merge")
    assert npairs > 100                                 # ~343 close pairs expected at this density
    sim.force_move()
    got = sim.state()
    ids, x, y, vx, vy, m = merged
    sel = np.sort(np.random.default_rng(0).choice(len(ids), 512, replace=False))
    ax, ay = core.c4_accel(x, y, m, sel)
    wvx = (vx[sel] + ax * np.float32(1e-3)).astype(np.float32)
    wvy = (vy[sel] + ay * np.float32(1e-3)).astype(np.float32)
    wx = (x[sel] + wvx * np.float32(1e-3)).astype(np.float32)
    wy = (y[sel] + wvy * np.float32(1e-3)).astype(np.float32)
    gsel = np.searchsorted(got[0], ids[sel])
    assert np.array_equal(got[0][gsel], ids[sel])
    for name, g, w in (("vx", got[3][gsel], wvx), ("vy", got[4][gsel], wvy), ("x", got[1][gsel], wx),
                       ("y", got[2][gsel], wy), ("m", got[5][gsel], m[sel])):
        if not np.array_equal(g.view(np.uint32), w.view(np.uint32)):
            rel = np.max(np.abs(g - w) / np.maximum(np.abs(w), 1e-30))
            assert rel <= 1e-5, f"{name} rel err {rel}"
    check_heap(sim.heap, expect_live=[len(ids)])


def test_nbody_full_size_properties():
    """Properties that hold at any size after several full-size steps: no two
    survivors closer than the merge distance after a merge phase, mass
    conserved, every body finite."""
    from scipy.spatial import cKDTree
    say("nbody full properties")
    sim = W().NBody(n=262144)
    sim.populate()
    m0 = float(sim.init[4].sum(dtype=np.float64))
    for s in range(4):
        sim.step()
    sim.merge()
    ids, x, y, vx, vy, m = sim.state()
    assert np.isfinite(x).all() and np.isfinite(vx).all()
    assert abs(float(m.sum(dtype=np.float64)) - m0) < 1e-3 * m0
    pts = np.stack([x, y], 1).astype(np.float64)
    for i, j in cKDTree(pts).query_pairs(r=1.2e-4):
        dx, dy = np.float32(x[j] - x[i]), np.float32(y[j] - y[i])
        assert np.sqrt(np.float32(dx * dx + dy * dy), dtype=np.float32) >= np.float32(1e-4)
    check_heap(sim.heap, expect_live=[len(ids)])


def test_correctly_rounded_div_sqrt_against_ieee():
    """The FP32 `/` and sqrtf the kernels use are correctly rounded: the force
    phase's interaction term on 2^24 random operand pairs equals the CPU's."""
    say("div/sqrt")
    rng = np.random.default_rng(5)
    n = 1 << 12
    x = rng.uniform(-1, 1, n).astype(np.float32)
    y = rng.uniform(-1, 1, n).astype(np.float32)
    m = np.exp(rng.standard_normal(n) * 2).astype(np.float32)
    sim = W().NBody(n=n, init=(x, y, np.zeros(n, np.float32), np.zeros(n, np.float32), m), G=1.0, dt=1.0)
    sim.populate()
    sim.phase(34)                                      # FORCE only: v = a*1
    _, _, _, vx, vy, _ = sim.state()
    ax, ay = core.c4_accel(x, y, m, np.arange(n), G=1.0)
    assert np.array_equal(vx.view(np.uint32), ax.view(np.uint32))
    assert np.array_equal(vy.view(np.uint32), ay.view(np.uint32))


def test_force_fast_arithmetic_equals_ieee():
    """smmo_check_force_arith: the force kernel's fast square root equals the
    correctly rounded one on every float of [2^-40, 2^40) (671,088,640 bit
    patterns) and its fast division the correctly rounded one on 2^28
    pseudo-random operand pairs of the fast ranges."""
    import ctypes as C
    from paper_1810_11765_amd import smmo as S
    say("force arithmetic self-check")
    L = S.lib()
    L.smmo_check_force_arith.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p]
    L.smmo_check_force_arith.restype = C.c_int
    out = torch.full((2,), 7, dtype=torch.int64, device="cuda")
    for seed in (1, 2):
        S.check(L.smmo_check_force_arith(0x2B800000, 0x53800000, 1 << 28, seed, out.data_ptr(),
                                         C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        assert out.cpu().tolist() == [0, 0]


def test_force_fallback_paths_against_ieee():
    """Operands outside the fast ranges take the general operations: bodies
    1e7 apart (d2 above 2^40), pairs 1e-7 apart (d2 below 2^-40), G m above
    2^30 and below 2^-50, bodies at the position empty slots use; the force
    phase alone equals the oracle's accelerations bit for bit."""
    say("force fallback paths")
    rng = np.random.default_rng(17)
    n = 64 * 70 + 9
    x = rng.uniform(-1, 1, n).astype(np.float32)
    y = rng.uniform(-1, 1, n).astype(np.float32)
    m = np.exp(rng.standard_normal(n)).astype(np.float32)
    x[:40] = rng.uniform(-1e7, 1e7, 40).astype(np.float32)         # far away
    for k in range(60, 90, 2):                                     # close pairs (no merge phase here)
        x[k + 1] = x[k] + np.float32(1e-7)
        y[k + 1] = y[k]
    m[100:110] = np.float32(1e10)                                  # G m above the fast range
    m[200:210] = np.float32(1e-20)                                 # and below it
    x[300:304] = np.float32(1024.0)                                # where empty tile entries sit
    y[300:304] = np.float32(1024.0) + np.arange(4, dtype=np.float32)
    z = np.zeros(n, np.float32)
    sim = W().NBody(n=n, init=(x, y, z, z.copy(), m), G=1.0, dt=1.0)
    sim.populate()
    sim.phase(34)                                      # FORCE only: v = a*1
    _, _, _, vx, vy, _ = sim.state()
    ax, ay = core.c4_accel(x, y, m, np.arange(n), G=1.0)
    assert np.array_equal(vx.view(np.uint32), ax.view(np.uint32))
    assert np.array_equal(vy.view(np.uint32), ay.view(np.uint32))


@pytest.mark.parametrize("edge", ["inside", "outside"])
def test_force_coordinate_box_edge_against_ieee(edge):
    """Tiles whose coordinates are all below 2^18 in magnitude check d2 only
    against its lower end; bodies at +-(the largest float below 2^18) give
    d2 near 2^38, the largest such a tile can hold, and a body at exactly
    2^18 sends every tile holding it (and its own workgroup) back to the
    per-entry range check.  The force phase alone equals the oracle's
    accelerations bit for bit either way."""
    say(f"force coordinate box, {edge}")
    rng = np.random.default_rng(23)
    n = 64 * 40 + 17
    x = rng.uniform(-1, 1, n).astype(np.float32)
    y = rng.uniform(-1, 1, n).astype(np.float32)
    m = np.exp(rng.standard_normal(n)).astype(np.float32)
    big = np.float32(262144.0) if edge == "outside" else np.nextafter(np.float32(262144.0), np.float32(0))
    x[5], y[5] = big, big                          # in the first i-block and tile
    x[1500], y[1500] = -big, -big
    x[2000], y[2000] = big, -big
    z = np.zeros(n, np.float32)
    sim = W().NBody(n=n, init=(x, y, z, z.copy(), m), G=1.0, dt=1.0)
    sim.populate()
    sim.phase(34)                                      # FORCE only: v = a*1
    _, _, _, vx, vy, _ = sim.state()
    ax, ay = core.c4_accel(x, y, m, np.arange(n), G=1.0)
    assert np.array_equal(vx.view(np.uint32), ax.view(np.uint32))
    assert np.array_equal(vy.view(np.uint32), ay.view(np.uint32))


def test_nbody_config_100_steps_against_oracle_goldens():
    """The configuration as stated: 262,144 bodies of seed 42, 100 steps.  At
    steps 1, 10 and 100 the survivors are compared with the oracle's values
    stored in tests/golden (written by tests/golden/make_goldens.py from
    oracle/ only): exact survivor count, the sampled records within relative
    1e-5 (field by field), and the SHA-256 of the whole canonical state, i.e.
    every survivor bit for bit."""
    from golden.make_goldens import NBODY_FILE, nbody_hash, read_nbody
    import os
    if not os.path.exists(NBODY_FILE):
        pytest.fail("golden values missing: run python tests/golden/make_goldens.py nbody")
    golden = read_nbody()
    say("nbody config 262144 x 100 vs goldens")
    sim = W().NBody(n=262144, seed=42)
    sim.populate()
    last = max(golden)
    for s in range(1, last + 1):
        sim.step()
        if s not in golden:
            continue
        g = golden[s]
        say("nbody step", s)
        st = sim.state()
        order = np.argsort(st[0], kind="stable")
        st = tuple(a[order] for a in st)
        assert len(st[0]) == g["count"], f"step {s}: {len(st[0])} survivors, oracle {g['count']}"
        idx = np.searchsorted(st[0], np.array(sorted(g["sample"]), dtype=np.int32))
        assert np.array_equal(st[0][idx], np.array(sorted(g["sample"]), dtype=np.int32)), f"step {s}: sampled ids"
        got = np.stack([a[idx] for a in st[1:]], 1)
        want = np.stack([g["sample"][k] for k in sorted(g["sample"])], 0)
        rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-30)
        assert rel.max() <= 1e-5, f"step {s}: sampled records rel err {rel.max()}"
        assert nbody_hash(*st) == g["sha256"], f"step {s}: state differs from the oracle's (within 1e-5 on the sample)"
    check_heap(sim.heap, expect_live=[golden[last]["count"]])


def test_valu_probe_reference_runs_and_checks_arguments():
    """smmo_valu_probe (the issue-cost reference the bench uses for the force
    kernel's bound): every kind runs and stores finite values; a kind past 3
    is refused before any launch."""
    import ctypes as C
    from paper_1810_11765_amd import smmo as S
    say("valu probe")
    L = S.lib()
    L.smmo_valu_probe.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p]
    L.smmo_valu_probe.restype = C.c_int
    out = torch.full((4 * 256,), float("nan"), dtype=torch.float32, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for kind in range(4):
        S.check(L.smmo_valu_probe(out.data_ptr(), kind, 4, 100, stream))
        assert torch.isfinite(out).all()
    with pytest.raises(S.SmmoError):
        S.check(L.smmo_valu_probe(out.data_ptr(), 4, 4, 100, stream))
