"""cloth_debug_candidates_noalloc (the broad-phase query on the library's fixed device
scratch, no device allocation) against cloth_debug_candidates (buffers allocated per call)
and against the FP32 brute force, through the C ABI: two calls in a row, the second over
fewer points, then the first again (the scratch keeps the last call's contents), plus the
size limits.  Integer results: bit-exact."""
import numpy as np
import pytest

import oracle
from paper_2507_11794_amd import cloth as B
from paper_2507_11794_amd import workloads as W

pytestmark = pytest.mark.gpu


def _points(inp, n, seed):
    rng = np.random.default_rng(seed)
    V = inp.verts.astype(np.float64)
    near = V[rng.integers(0, V.shape[0], n - n // 8)] + rng.normal(0, 0.008, size=(n - n // 8, 3))
    far = rng.uniform(-2, 2, size=(n // 8, 3))
    return np.concatenate([near, far]).astype(np.float32)


def test_noalloc_candidates_equal_the_allocating_query_on_consecutive_calls():
    inp = W.config1(n=20, freq=24)
    big, small = _points(inp, 6000, 1), _points(inp, 900, 2)
    with B.Cloth(inp) as sim:
        ref_big, ref_small = sim.debug_candidates(big), sim.debug_candidates(small)
        got_big = sim.debug_candidates(big, noalloc=True)
        got_small = sim.debug_candidates(small, noalloc=True)
        again = sim.debug_candidates(big, noalloc=True)
    print(f"{big.shape[0]} points: {ref_big.shape[0]} pairs; {small.shape[0]} points: "
          f"{ref_small.shape[0]} pairs")
    assert ref_big.shape[0] > 1000 and ref_small.shape[0] > 100
    assert np.array_equal(got_big, ref_big)
    assert np.array_equal(got_small, ref_small)
    assert np.array_equal(again, ref_big)
    assert np.array_equal(ref_small, oracle.candidates_f32(small, inp.verts, inp.tris,
                                                           inp.thickness))


def test_noalloc_candidates_limits_and_counts():
    import ctypes as C
    inp = W.small_collision_scene(n=8, freq=3)
    lib = B.load()
    with B.Cloth(inp) as sim:
        # more points than the scratch takes: refused before any device work
        P = np.zeros((65537, 3), dtype=np.float32)
        n = C.c_longlong(-1)
        st = lib.cloth_debug_candidates_noalloc(C.c_void_p(sim.h), P.shape[0],
                                                P.ctypes.data_as(C.POINTER(C.c_float)), None, 0,
                                                C.byref(n))
        assert st == B.CLOTH_ENOMEM and n.value == 0
        # the largest accepted call, count only (cap 0): the same total as the allocating query
        P = _points(inp, 65536, 3)
        n = C.c_longlong(-1)
        st = lib.cloth_debug_candidates_noalloc(C.c_void_p(sim.h), P.shape[0],
                                                P.ctypes.data_as(C.POINTER(C.c_float)), None, 0,
                                                C.byref(n))
        assert st == B.CLOTH_OK
        assert n.value == sim.debug_candidates(P).shape[0]
        # zero points: nothing to do
        n = C.c_longlong(-1)
        assert lib.cloth_debug_candidates_noalloc(C.c_void_p(sim.h), 0, None, None, 0,
                                                  C.byref(n)) == B.CLOTH_OK and n.value == 0
