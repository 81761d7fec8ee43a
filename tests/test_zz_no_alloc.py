"""smmo_parallel_do_static_scratch (the entry point that allocates nothing):
through the C-ABI, its results equal smmo_parallel_do's on the same inputs,
call after call, the second input smaller than the first."""
import functools

import numpy as np
import pytest

from helpers import check_heap, say
from oracle import core

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _static(heap):
    """Route every do-all of `heap` through smmo_parallel_do_static_scratch."""
    heap.parallel_do = functools.partial(heap.parallel_do, static_scratch=True)


def test_static_scratch_do_all_equals_the_heap_scratch_form():
    from paper_1810_11765_amd import smmo as S
    from paper_1810_11765_amd import workloads as W
    # call 1: predator-prey in a 300,000-block heap, so every do-all builds its
    # block list through level 1 (staged in the static scratch), 25 steps
    side, seed, steps = 150, 31, 25
    ref = W.WaTor(seed=seed, width=side, height=side, num_blocks=300_000)
    st = W.WaTor(seed=seed, width=side, height=side, num_blocks=300_000, kind0=ref.kind0)
    _static(st.heap)
    for w in (ref, st):
        w.populate()
    say("static scratch: predator-prey", side, "in 300000 blocks", steps, "steps")
    for _ in range(steps):
        ref.step()
        st.step()
    a, b = ref.state(), st.state()
    assert all(np.array_equal(x, y) for x, y in zip(a, b)), "static-scratch do-alls differ from the heap-scratch ones"
    ok, oa, oe = core.c3_run(ref.kind0, side, side, seed, steps)
    assert np.array_equal(b[0], ok) and np.array_equal(b[1][ok > 0], oa[ok > 0])
    check_heap(st.heap, expect_live=[int((ok == 1).sum()), int((ok == 2).sum())])
    ref.heap.close(); st.heap.close()
    # call 2, smaller: n-body with merging, 3,000 bodies, 3 steps (the force's
    # ordered block list in the static scratch, whose counters still hold the
    # values of call 1)
    say("static scratch: n-body 3000 x 3")
    init = None
    sims = []
    for static in (False, True):
        nb = W.NBody(n=3000, seed=9, G=1e-4, init=init)
        init = nb.init
        if static:
            _static(nb.heap)
        nb.populate()
        for _ in range(3):
            nb.step()
        sims.append(nb.state())
    for x, y in zip(*sims):
        assert np.array_equal(np.asarray(x).view(np.uint8), np.asarray(y).view(np.uint8))
    # call 3, smaller again: a do-all on an 8-block heap
    say("static scratch: visit in 8 blocks")
    h = S.Heap([[4]], 8)
    n = 8 * 64 - 5
    ids = torch.arange(n, dtype=torch.int32, device="cuda")
    h.parallel_new(0, n, S.CTOR_ARRAYS, S.ctor_arrays([ids]))
    visits = torch.zeros(n, dtype=torch.int32, device="cuda")
    h.parallel_do(0, S.M_VISIT, S.VisitArgs(visits.data_ptr()), static_scratch=True)
    assert (visits.cpu().numpy() == 1).all()


def test_static_scratch_rejects_heaps_above_its_limit():
    from paper_1810_11765_amd import smmo as S
    h = S.Heap([[1]], (1 << 20) + 1)
    with pytest.raises(S.SmmoError):
        h.parallel_do(0, S.M_DESTROY_ALL, static_scratch=True)
    h.close()
