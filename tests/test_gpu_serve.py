"""GPU serving: requests admitted while others run give results identical to
solo runs (continuous batching, mixed storage types, memory budget)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (run with -m 'not gpu' on CPU)")
    from paper_2009_04619_amd import wave
    return wave


def test_served_results_equal_solo_runs(W):
    from paper_2009_04619_amd.serve import GpuExecutor, Request, Server, summarize
    rng = np.random.default_rng(7)
    reqs = []
    for q in range(8):
        nx, ny, nz = (int(v) for v in rng.choice([48, 64, 80, 96], 3))
        steps = int(rng.integers(20, 60))
        s = synth.config_small_layered(nx, ny, nz, 6, steps, seed=900 + q)
        reqs.append(Request(rid=q, arrival=0.02 * q, shot=s, storage=["f32", "bf16", "f16"][q % 3]))
    ex = GpuExecutor(graph_steps=0)
    budget = 3 * max(ex.bytes_for(r) for r in reqs)      # at most ~3 resident
    srv = Server(ex, budget_bytes=budget, block_steps=7)
    done = srv.run(reqs, keep_fields=set(range(8)))
    ex.close()
    print(summarize(done, max(r.finished for r in done)), flush=True)
    assert srv.peak_in_use <= budget
    admit = {e[1]: e[2] for e in srv.log if e[0] == "admit"}
    fin = {e[1]: e[2] for e in srv.log if e[0] == "finish"}
    assert any(admit[b] < fin[a] and admit[a] < admit[b] for a in fin for b in fin)  # overlap
    for r in done:
        assert r.error is None
        sh = W.shot_from_synth(r.shot, storage=r.storage)
        sh.step(r.shot.steps)
        assert np.array_equal(sh.read(W.WAVE_FIELD_U), r.field), r.rid
        assert np.array_equal(sh.traces(), r.traces), r.rid
        sh.close()
