"""GPU serving: requests admitted while others run give results identical to
solo runs (continuous batching, mixed storage types, memory budget), and
each within its storage type's bound of the float64 oracle."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (run with -m 'not gpu' on CPU)")
    from paper_2009_04619_amd import wave
    return wave


def rel_l2(a, b):
    n = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / n) if n > 0 else float(np.linalg.norm(a))


def bound(storage, steps):
    """Relative L2 bound against float64: 1e-5 for float32 storage; for
    16-bit storage 2 sqrt(N) u, u the storage rounding unit (one rounding per
    stored value and step, accumulating like a random walk)."""
    if storage == "f32":
        return 1e-5
    return 2.0 * np.sqrt(steps) * (2.0 ** -8 if storage == "bf16" else 2.0 ** -11)


# smallest normal number of each storage format
TINY = {"f32": 2.0 ** -126, "bf16": 2.0 ** -126, "f16": 2.0 ** -14}


def test_served_results_equal_solo_runs(W):
    from paper_2009_04619_amd.serve import GpuExecutor, Request, Server, summarize
    rng = np.random.default_rng(7)
    reqs = []
    for q in range(8):
        nx, ny, nz = (int(v) for v in rng.choice([48, 64, 80, 96], 3))
        steps = int(rng.integers(20, 60))
        s = synth.config_small_layered(nx, ny, nz, 6, steps, seed=900 + q)
        # all arrive at once, so that several are resident together however
        # fast each one runs (the budget admits about three at a time)
        reqs.append(Request(rid=q, arrival=0.0, shot=s, storage=["f32", "bf16", "f16"][q % 3]))
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
    worst = {}
    for r in done:
        assert r.error is None
        sh = W.shot_from_synth(r.shot, storage=r.storage)
        sh.step(r.shot.steps)
        assert np.array_equal(sh.read(W.WAVE_FIELD_U), r.field), r.rid
        assert np.array_equal(sh.traces(), r.traces), r.rid
        sh.close()
        # error of the served result against the float64 oracle, within the
        # stated bound of its storage type
        o = oracle.run_shot(r.shot, precision="f64")
        ef = rel_l2(r.field, o["u"])
        # traces: receivers whose signal is inside the storage format's normal
        # range (binary16 flushes amplitudes below 2^-14, e.g. the stencil's
        # precursors ahead of a wavelet that has barely started)
        keep = np.abs(o["traces"]).max(axis=0) >= TINY[r.storage]
        et = rel_l2(r.traces[:, keep], o["traces"][:, keep]) if keep.any() else 0.0
        assert max(ef, et) < bound(r.storage, r.shot.steps), (r.rid, r.storage, ef, et)
        worst[r.storage] = max(worst.get(r.storage, 0.0), ef, et)
    print("served results, max rel L2 vs float64 per storage:",
          {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
