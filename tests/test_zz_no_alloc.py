"""numa_step_batch_noalloc (static device scratch, no allocation) against
numa_step_batch (caller scratch) through the C ABI.

Both run the same kernels on the same per-item code, so the results must be
bitwise equal.  Two calls in a row, the second with a smaller input, check
that the shared static array carries nothing from one call into the next.
"""
import numpy as np
import pytest

from paper_1511_01561_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def box(n, N, seed, nz):
    Lx, H = n * 6250.0, nz * 1250.0
    rng = np.random.default_rng(seed)
    c = (rng.uniform(0, Lx), rng.uniform(0, Lx), rng.uniform(0.25 * H, 0.75 * H))
    return inputs.box_workload(n, n, nz, N, Lx, Lx, H, terrain=500.0, bubble_centre=c,
                               bubble_amp=rng.uniform(0.1, 2.0))


def make(wl, seed, stage=None):
    from paper_1511_01561_amd import numa
    g = numa.Mesh(wl["mesh"], wl["phys"], prec_mask=3)
    g.set_metric(numa.METRIC_RECOMPUTE)
    if stage is not None:
        g.set_stage(stage)
    return g, g.init_state(wl["ic"], inputs.device_noise(g.n_unique, seed))


def run_both(torch, objs, prec, nsteps, dt=0.05):
    """the noalloc call on clones of the states, numa_step_batch on others"""
    from paper_1511_01561_amd import numa
    qa = [q.clone() for _, q in objs]
    qb = [q.clone() for _, q in objs]
    print("noalloc: %d items, prec %d, %d steps" % (len(objs), prec, nsteps), flush=True)
    numa.step_batch_noalloc([(g, q, dt) for (g, _), q in zip(objs, qa)], nsteps, prec)
    numa.step_batch([(g, q, numa.alloc_scratch(g, prec), dt) for (g, _), q in zip(objs, qb)], nsteps, prec)
    torch.cuda.synchronize()
    return qa, qb


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_equals_step_batch_twice(torch_cuda, prec):
    from paper_1511_01561_amd import numa
    torch = torch_cuda
    numa.step_batch_noalloc([], 0, prec)  # set-up on this device
    # first call: three items of different sizes and stage modes
    big = [make(box(8, 4, 1, 4), 11), make(box(8, 4, 2, 4), 12, numa.STAGE_BLOCK),
           make(box(4, 4, 3, 2), 13, numa.STAGE_COLOUR)]
    qa, qb = run_both(torch, big, prec, 3)
    for (_, q0), a, b in zip(big, qa, qb):
        assert torch.equal(a, b)
        assert not torch.equal(a, q0)
    # second call: one smaller item, which reuses the start of the array
    small = [make(box(4, 4, 4, 2), 14)]
    qa, qb = run_both(torch, small, prec, 2, dt=0.07)
    assert torch.equal(qa[0], qb[0])
    assert not torch.equal(qa[0], small[0][1])


def test_noalloc_flags_and_graph_capture(torch_cuda):
    """the non-finite flag reaches the caller, and a captured noalloc call
    replays like the eager one"""
    from paper_1511_01561_amd import numa
    torch = torch_cuda
    objs = [make(box(4, 4, 5, 2), 15), make(box(4, 4, 6, 2), 16)]
    objs[1][1][1, 7] = float("nan")
    flags = torch.zeros(2, dtype=torch.int32, device="cuda:0")
    qa = [q.clone() for _, q in objs]
    numa.step_batch_noalloc([(g, q, 0.05, flags[k:k + 1]) for k, ((g, _), q) in enumerate(zip(objs, qa))], 1, 0)
    torch.cuda.synchronize()
    assert flags.tolist() == [0, 1]
    # graph: capture one step on a side stream, replay it three times
    ref = [objs[0][1].clone()]
    qg = [objs[0][1].clone()]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        h = numa.lib()
        import ctypes as ct
        arr = numa._items([(objs[0][0], qg[0], None, 0.05)])
        st = ct.c_void_p(s.cuda_stream)
        numa.check(h.numa_step_batch_noalloc(arr, 1, 0, 0, st))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
            numa.check(h.numa_step_batch_noalloc(arr, 1, 0, 1, st))
    for r in range(3):
        g.replay()
        torch.cuda.synchronize()
        numa.step_batch([(objs[0][0], ref[0], numa.alloc_scratch(objs[0][0], 0), 0.05)], 1, 0)
        torch.cuda.synchronize()
        assert torch.equal(qg[0], ref[0]), r


def test_noalloc_rejects_what_does_not_fit(torch_cuda):
    from paper_1511_01561_amd import numa
    torch = torch_cuda
    g, q = make(box(16, 4, 7, 16), 17)
    per = numa.step_scratch_bytes(g, 0)
    fit = numa.NOALLOC_SCRATCH_BYTES // per
    assert 1 <= fit < 8
    qs = [q.clone() for _ in range(fit + 1)]
    q0 = [x.clone() for x in qs]
    with pytest.raises(numa.NumaError, match="error -2.*static scratch holds %d" % numa.NOALLOC_SCRATCH_BYTES):
        numa.step_batch_noalloc([(g, x, 0.05) for x in qs], 1, 0)
    g2, q2 = make(box(4, 4, 8, 2), 18)
    many = [q2.clone() for _ in range(numa.NOALLOC_MAX_ITEMS + 1)]
    with pytest.raises(numa.NumaError, match="at most %d" % numa.NOALLOC_MAX_ITEMS):
        numa.step_batch_noalloc([(g2, x, 0.05) for x in many], 1, 0)
    scr = numa.alloc_scratch(g2, 0)
    with pytest.raises(numa.NumaError, match="library supplies the scratch"):
        numa.check(numa.lib().numa_step_batch_noalloc(numa._items([(g2, many[0], scr, 0.05)]), 1, 0, 1,
                                                       numa._stream(None)))
    torch.cuda.synchronize()
    for a, b in zip(qs, q0):  # nothing ran
        assert torch.equal(a, b)
    # the largest batch that fits runs and matches numa_step_batch
    qa, qb = run_both(torch, [(g, x) for x in q0[:fit]], 0, 1)
    for a, b in zip(qa, qb):
        assert torch.equal(a, b)
