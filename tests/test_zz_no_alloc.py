"""GPU: pp_batch_step_noalloc, the batch step whose descriptor tables live in the library's
static device array, gives bitwise the results of pp_batch_step (the same kernels; the tables
only sit elsewhere).  Two phases in a row on the same process: a batch of four runs of
different boxes, field orders and pushers, then a smaller batch of one small run, so the second
phase reads tables written over the first phase's larger ones.  A batch whose tables exceed
the static array is refused with PP_E_CAPACITY and nothing enqueued, while pp_batch_step still
steps it."""
import sys

import numpy as np
import pytest

from test_gpu_batch import RUNS, _assert_same, _make, _state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ppm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1211_4575_amd import pp
    pp.lib()
    return pp


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _step_batch(ppm, runs, steps, noalloc):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    batch = ppm.pp_batch_create(8, stream)
    try:
        for r in runs:
            ppm.pp_batch_add(batch, r.handle)
        for _ in range(steps):
            if noalloc:
                ppm.pp_batch_step_noalloc(batch)
            else:
                ppm.pp_batch_step(batch)
    finally:
        ppm.pp_batch_destroy(batch)
    out = []
    for r in runs:
        d = r.diagnostics(ppm.PP_DIAG_MOMENTS)
        assert d.flags == 0 and d.step == steps
        out.append(_state(r))
        r.close()
    return out


@pytest.mark.parametrize("O", [2, 3], ids=["quadratic", "cubic"])
def test_noalloc_step_equals_step_larger_then_smaller(ppm, orc, O):
    for phase, (members, steps) in enumerate(((tuple(range(len(RUNS))), 3), ((3,), 2))):
        _say("no-alloc phase", phase, "members", members, "steps", steps, "order", O)
        ref = _step_batch(ppm, [_make(ppm, orc, k, O) for k in members], steps, noalloc=False)
        got = _step_batch(ppm, [_make(ppm, orc, k, O) for k in members], steps, noalloc=True)
        for k, a, b in zip(members, got, ref):
            _assert_same(a, b, f"phase {phase} run {k}")


def test_noalloc_step_refuses_tables_beyond_the_static_array(ppm):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(5)
    n = (4, 4, 4)
    P = ppm.make_params(n=n, shape_order=3, field_order=2, precision=ppm.PP_PREC_FP32_SPLIT)
    runs = []
    batch = ppm.pp_batch_create(4096, stream)
    refused_at = None
    try:
        # add one-species 4^3 runs until the tables no longer fit (bounded: 3000 runs)
        for k in range(3000):
            cell = rng.integers(0, 64, 64).astype(np.int32)
            off = rng.uniform(0.0, 1.0, (3, 64)).astype(np.float32)
            u = rng.normal(0.0, 0.05, (3, 64)).astype(np.float32)
            runs.append(ppm.Run(P, [dict(q=-1.0, m=1.0, w=1.0, cell=cell, off=off, u=u)], with_id=False))
            ppm.pp_batch_add(batch, runs[-1].handle)
            if k % 64 == 63 or k == 2999:
                try:
                    ppm.pp_batch_step_noalloc(batch)
                except ppm.PPError as e:
                    assert e.status == ppm.PP_E_CAPACITY, str(e)
                    assert "static" in str(e), str(e)
                    refused_at = k + 1
                    break
        _say("static table array refused", refused_at, "runs")
        assert refused_at is not None, "3000 runs still fit the static table array"
        steps_before = [r.diagnostics(ppm.PP_DIAG_MOMENTS).step for r in runs]
        ppm.pp_batch_step(batch)  # the growable tables still take them
        steps_after = [r.diagnostics(ppm.PP_DIAG_MOMENTS).step for r in runs]
        assert all(b == a + 1 for a, b in zip(steps_before, steps_after))
    finally:
        ppm.pp_batch_destroy(batch)
        for r in runs:
            r.close()
