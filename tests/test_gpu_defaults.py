"""The launch mapping smnn_plan_create picks when the caller leaves the chunk
lengths at 0 (plans only, no solve).

Rules under test:
- level 0: 4 for 3 x 3 and 4 x 4 blocks in the FP64 I/O modes; with float
  I/O 8 from 2^22 steps per batch on, else 4;
- separator levels: 8, except for 3 x 3 blocks where chunks of 4 let the
  single upper-level launch start at the same level as chunks of 8 would;
- that launch starts at the first level >= 1 that is not the last, where
  every instance has at most 64 chunks (3 x 3 blocks) and the level holds
  at most 2^19 nodes.
The expected values below are worked out by hand in the comments.
"""
import pytest

pytestmark = pytest.mark.gpu


def _plan(order, n_inst, steps, mode, **kw):
    from paper_2410_06074_amd import Plan
    return Plan(order=order, n_init=order, n_inst=n_inst, steps=steps, mode=mode, **kw)


CASES = [
    # 1536 x 1,000, R = 2: level 1 has 249 nodes per instance (382,464 in all).
    # Chunks of 8 there: 32 per instance; of 4: 63 <= 64, so both start at
    # level 1 and 4 is taken.
    (2, 1536, 1000, "fp64r", 4, 4, 1),
    (2, 1536, 1000, "fp64", 4, 4, 1),
    # float I/O, 1.5e6 steps < 2^22: level-0 chunks of 4, then as above
    (2, 1536, 1000, "fp32r", 4, 4, 1),
    # 1536 x 10,000: level 1 has 2,499 nodes per instance.  Chunks of 8:
    # level 2 has 312 (39 chunks, 479,232 nodes) -> start 2.  Chunks of 4:
    # level 2 has 624 (156 chunks), level 3 155 (39 chunks) -> start 3 > 2,
    # so 8 stays.
    (2, 1536, 10000, "fp64r", 4, 8, 2),
    # float I/O, 1.5e7 steps: level-0 chunks of 8, level 1 1,249 nodes;
    # chunks of 8 start at level 2 (156 nodes, 20 chunks), chunks of 4 at 3
    (2, 1536, 10000, "fp32r", 8, 8, 2),
    # 4096 x 1,460, float I/O (6.0e6 steps): level 1 has 182 nodes per
    # instance, 745,472 in all (> 2^19).  Chunks of 8: level 2 has 22 nodes
    # (3 chunks) and a level 3 -> start 2.  Chunks of 4: level 2 has 45 nodes
    # (12 chunks, 184,320 in all) and a level 3 -> start 2 as well: 4.
    (2, 4096, 1460, "fp32r", 8, 4, 2),
    # R = 3 (4 x 4 blocks): the separator chunk rule is for 3 x 3 blocks only
    (3, 1536, 1000, "fp64r", 4, 8, None),
]


@pytest.mark.parametrize("order,n_inst,steps,mode,chunk,upper,top", CASES)
def test_default_chunks(order, n_inst, steps, mode, chunk, upper, top):
    p = _plan(order, n_inst, steps, mode)
    assert (p.chunk, p.chunk_upper) == (chunk, upper)
    if top is not None:
        assert p.top_level == top


@pytest.mark.parametrize("steps,chunk", [(1 << 22, 8), ((1 << 22) - 1, 4)])
def test_float_io_level0_chunk_threshold(steps, chunk):
    # one instance of 2^22 steps (the threshold) and one step fewer
    assert _plan(2, 1, steps, "fp32r").chunk == chunk


def test_explicit_chunks_are_kept():
    p = _plan(2, 1536, 1000, "fp64r", chunk_upper=8)
    assert (p.chunk, p.chunk_upper) == (4, 8)
    assert p.top_level == 1     # 32 chunks of 8 per instance at level 1
    p = _plan(2, 1536, 1000, "fp32r", chunk=8)
    assert p.chunk == 8
