"""GPU batching: several shots advanced by one sweep launch per step.

Every member must end bit for bit where it ends when stepped on its own
(same per-point arithmetic, same order), whether the steps run as plain
launches or as replays of a captured graph, and across membership changes.
"""
import sys

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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


SHAPES = [  # nx, ny, nz, w, steps, storage
    (70, 45, 37, 5, 23),
    (128, 48, 64, 8, 30),
    (33, 90, 41, 4, 7),
    (64, 64, 64, 16, 30),
    (150, 20, 18, 3, 12),
]


def shots_for(shapes, seed0=100):
    out = []
    for q, (nx, ny, nz, w, steps) in enumerate(shapes):
        out.append(synth.config_small_layered(nx, ny, nz, w, steps, seed=seed0 + q, nsrc=1 + q % 2))
    return out


def read_all(W, sh):
    return dict(u=sh.read(W.WAVE_FIELD_U), u_prev=sh.read(W.WAVE_FIELD_UPREV),
                phi=sh.read(W.WAVE_FIELD_PHI), traces=sh.traces(), n=sh.step_count)


def solo(W, s, storage="f32"):
    sh = W.shot_from_synth(s, storage=storage)
    sh.step(s.steps)
    r = read_all(W, sh)
    sh.close()
    return r


def rel_l2(a, b):
    n = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / n) if n > 0 else float(np.linalg.norm(a))


def same(a, b, what):
    assert a["n"] == b["n"], what
    for k in ("u", "u_prev", "phi", "traces"):
        assert a[k].shape == b[k].shape, (what, k)
        assert np.array_equal(a[k], b[k]), (what, k, int((a[k] != b[k]).sum()))


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("graph", [0, 4])
@pytest.mark.parametrize("tile", [(1, 16), (2, 16)])
def test_batch_members_equal_solo_runs(W, storage, graph, tile):
    shots = shots_for(SHAPES)
    say(f"case batch storage={storage} graph={graph} tile={tile}")
    ref = [solo(W, s, storage) for s in shots]
    b = W.Batch(storage=storage, max_shots=8)
    b.set_kernel(*tile)
    b.set_graph(graph)
    members = []
    for s in shots:
        sh = W.shot_from_synth(s, storage=storage)
        b.add(sh, s.steps)
        members.append(sh)
    for n in (10, 1, 9, 20):          # uneven runs; members stop at their own count
        b.run(n)
    for s, sh in zip(shots, members):
        assert b.remaining(sh) == 0
    got = [read_all(W, sh) for sh in members]
    for q, (g, r) in enumerate(zip(got, ref)):
        same(g, r, f"member {q}")
    b.close()
    for sh in members:
        sh.close()
    # and one member against the oracle directly
    o = oracle.run_shot(shots[1], precision="f32", storage=storage)
    assert np.array_equal(got[1]["u"], o["u"]) and np.array_equal(got[1]["traces"], o["traces"])
    # every member against float64, within its storage type's bound
    worst = 0.0
    for q, (g, s) in enumerate(zip(got, shots)):
        o64 = oracle.run_shot(s, precision="f64")
        err = max(rel_l2(g["u"], o64["u"]), rel_l2(g["traces"], o64["traces"]))
        lim = 1e-5 if storage == "f32" else 2.0 * np.sqrt(s.steps) * 2.0 ** -8
        assert err < lim, (q, storage, err, lim)
        worst = max(worst, err)
    say(f"batch {storage}: max rel L2 vs float64 over members {worst:.2e}")


def test_graph_replays_match_plain_launches_across_runs(W):
    shots = shots_for(SHAPES[:3], seed0=200)
    for s in shots:
        s.steps = 40
        s.wavelet = np.ascontiguousarray(np.pad(s.wavelet, ((0, 0), (0, 40))))[:, :40]
    say("case graph replay vs plain")
    runs = {}
    for graph in (0, 5):
        b = W.Batch(max_shots=4)
        b.set_graph(graph)
        members = [W.shot_from_synth(s) for s in shots]
        for s, sh in zip(shots, members):
            b.add(sh, 40)
        snaps = []
        for _ in range(4):             # 4 runs of 10 steps: 2 graph replays each
            b.run(10)
            snaps.append([read_all(W, sh) for sh in members])   # host reads in between
        runs[graph] = snaps
        b.close()
        for sh in members:
            sh.close()
    for t in range(4):
        for q in range(3):
            same(runs[5][t][q], runs[0][t][q], f"run {t} member {q}")


def test_membership_changes(W):
    shots = shots_for(SHAPES[:4], seed0=300)
    say("case membership changes")
    ref = [solo(W, s) for s in shots]
    b = W.Batch(max_shots=4)
    m = [W.shot_from_synth(s) for s in shots]
    b.add(m[0], shots[0].steps)
    b.add(m[1], shots[1].steps)
    b.run(5)
    b.add(m[2], shots[2].steps)       # joins while others are midway
    b.run(3)
    b.remove(m[1])                    # leaves midway, finishes on its own
    m[1].step(shots[1].steps - 8)
    b.add(m[3], shots[3].steps)
    b.run(100)
    for q in (0, 2, 3):
        same(read_all(W, m[q]), ref[q], f"member {q}")
    same(read_all(W, m[1]), ref[1], "member 1 (left)")
    b.close()
    for sh in m:
        sh.close()


def test_batch_error_paths(W):
    s = shots_for(SHAPES[:1])[0]
    b = W.Batch(storage="f32", max_shots=1)
    sh = W.shot_from_synth(s)
    other = W.shot_from_synth(s, storage="bf16")
    assert W.wave_batch_add(b.b, other.ctx, 5) == W.WAVE_EINVAL      # storage differs
    assert W.wave_batch_add(b.b, sh.ctx, s.steps + 1) == W.WAVE_EINVAL  # traces overflow
    assert W.wave_batch_add(b.b, sh.ctx, 5) == W.WAVE_OK
    assert W.wave_batch_add(b.b, sh.ctx, 5) == W.WAVE_EINVAL          # already a member
    assert W.wave_step(sh.ctx, 1) == W.WAVE_EINVAL                    # stepped by the batch
    assert W.wave_batch_set_kernel(b.b, 3, 3) == W.WAVE_EINVAL
    assert W.wave_batch_run(b.b, -1) == W.WAVE_EINVAL
    b.close()
    assert W.wave_step(sh.ctx, 1) == W.WAVE_OK                        # free again
    sh.close()
    other.close()


def test_tuned_runs_stay_exact(W):
    """Tuning trials are ordinary steps: a tuned shot and a tuned batch end
    exactly where untuned runs end."""
    shots = shots_for(SHAPES[:3], seed0=400)
    n = 100                           # room for every candidate's trial steps
    for s in shots:
        s.steps = n
        s.wavelet = np.ascontiguousarray(np.pad(s.wavelet, ((0, 0), (0, n))))[:, :n]
    say("case tuned runs")
    ref = [solo(W, s) for s in shots]
    sh = W.shot_from_synth(shots[0])
    cfg = sh.tune(2)                  # ~20 candidates x (1 + 2) steps
    assert len(cfg) == 4 and sh.step_count < n
    sh.step(n - sh.step_count)
    same(read_all(W, sh), ref[0], "tuned shot")
    sh.close()
    b = W.Batch(max_shots=4)
    m = [W.shot_from_synth(s) for s in shots]
    for s, x in zip(shots, m):
        b.add(x, n)
    bc = b.tune(3)                    # 6 shapes x 3 steps
    assert len(bc) == 2
    b.run(2 * n)
    for q in range(3):
        same(read_all(W, m[q]), ref[q], f"tuned batch member {q}")
    b.close()
    for x in m:
        x.close()


def test_members_on_another_stream(W):
    """Members set up on a stream other than the batch's: the batch waits for
    their set-up, and a member that leaves waits for the runs it took part in
    before its own next step and reads."""
    import torch
    shots = shots_for(SHAPES[:3], seed0=500)
    say("case members on another stream")
    ref = [solo(W, s) for s in shots]
    side = torch.cuda.Stream()
    b = W.Batch(max_shots=4)
    m = [W.shot_from_synth(s, stream=side) for s in shots]
    for s, x in zip(shots, m):
        b.add(x, s.steps)
    b.run(7)
    b.remove(m[0])                    # leaves midway, continues on the side stream
    m[0].step(shots[0].steps - 7)
    b.run(100)
    for q in range(3):
        same(read_all(W, m[q]), ref[q], f"member {q}")
    b.close()
    for x in m:
        x.close()


@pytest.mark.parametrize("storage,tile", [("bf16", (0, 8)), ("f32", (0, 16))])
def test_batch_two_points_per_lane(W, storage, tile):
    """The batch on the two-points-per-lane kernel (rows_per_wave 0): members
    equal solo runs bit for bit, plain launches and captured blocks; the
    mode refuses members with an eta array."""
    shots = shots_for(SHAPES)
    say(f"case batch two points per lane storage={storage} tile={tile}")
    ref = [solo(W, s, storage) for s in shots]
    b = W.Batch(storage=storage, max_shots=8)
    assert W.wave_batch_set_kernel(b.b, 0, 12) == W.WAVE_EINVAL
    b.set_kernel(*tile)
    b.set_graph(4)
    members = []
    for s in shots:
        sh = W.shot_from_synth(s, storage=storage)
        b.add(sh, s.steps)
        members.append(sh)
    for n in (7, 1, 30):
        b.run(n)
    for q, (sh, r) in enumerate(zip(members, ref)):
        same(read_all(W, sh), r, f"pair member {q}")
    s0 = shots[0]
    _, e32 = oracle.eta_default(s0.nx, s0.ny, s0.nz, s0.w, s0.dx, s0.dy, s0.dz, s0.dt,
                                float(s0.vel.max()))
    with_eta = W.shot_from_synth(s0, storage=storage, eta=e32)
    assert W.wave_batch_add(b.b, with_eta.ctx, 5) == W.WAVE_EINVAL
    with_eta.close()
    b.close()
    for sh in members:
        sh.close()


def test_member_sources_and_receivers_are_fixed_while_in_a_batch(W):
    """A batch copies its members' source and receiver tables when they
    join, so adding a source or replacing the receivers of a member is
    refused (EINVAL) until it leaves; after leaving, the context takes both
    and ends where the oracle does."""
    say("case member source/receiver guard")
    s = synth.config_small_layered(70, 45, 37, 5, 12, seed=301, nsrc=1)
    sh = W.Shot(s.nx, s.ny, s.nz, s.w, s.dx, s.dy, s.dz, s.dt, s.vel, max_src=2,
                max_rec=len(s.rec), max_steps=s.steps)
    sh.inject(*s.src[0], s.wavelet[0])
    sh.record(s.rec)
    b = W.Batch(storage="f32", max_shots=2)
    b.add(sh, 6)
    b.run(6)
    extra = synth.ricker(s.steps, s.dt, t0=0.25 / 15.0)
    assert W.wave_inject(sh.ctx, 10, 11, 12, extra) == W.WAVE_EINVAL
    assert W.wave_record(sh.ctx, s.rec[:3]) == W.WAVE_EINVAL
    b.remove(sh)
    assert W.wave_inject(sh.ctx, 10, 11, 12, extra) == W.WAVE_OK
    sh.step(6)
    got = read_all(W, sh)
    b.close()
    sh.close()
    ref6 = oracle.run_shot(s, steps=6, precision="f32")
    s2 = synth.config_small_layered(70, 45, 37, 5, 12, seed=301, nsrc=1)
    s2.src = list(s.src) + [(10, 11, 12)]
    s2.wavelet = np.stack([s.wavelet[0], extra])
    ref = oracle.run_shot(s2, steps=6, precision="f32", n0=6,
                          state=dict(u=ref6["u"], u_prev=ref6["u_prev"], phi=ref6["phi"]))
    assert np.array_equal(got["u"], ref["u"])
    assert np.array_equal(got["traces"][6:], ref["traces"])
