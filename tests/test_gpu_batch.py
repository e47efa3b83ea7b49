"""Batched advance (one graph launch per RK substage over many uneven 2D
problems) against the same problems advanced one by one through the
single-grid calls: the states and times must agree bit for bit, for every
form, whatever the tile choice, with graphs or direct launches."""
import numpy as np
import pytest

from paper_2007_14933_amd import inputs as I
from parity_util import say

pytestmark = pytest.mark.gpu


def ensemble(sizes, seed, t_ends, scheme=I.TENO5):
    rng = np.random.default_rng(seed)
    return [I.riemann2d(n, rng, t_end=te, scheme=scheme) for n, te in zip(sizes, t_ends)]


SIZES = (32, 48, 24, 64, 40, 56)
T_ENDS = (0.02, 0.035, 0.01, 0.03, 0.025, 0.015)   # uneven: problems finish at different steps


def jump_sensor_bits():
    """A hand-set network that calls an interface smooth unless one of its
    six log-jump features is sizeable: z = 4 - 40 relu(relu(sum of jumps))."""
    from paper_2007_14933_amd import sensor as SN
    w = np.zeros(1441, dtype=np.float32)
    for i in range(4, 10):
        w[i * 32 + 0] = 1.0      # W1[i][0]
    w[352 + 0] = 1.0             # W2[0][0]
    w[1408 + 0] = -40.0          # w3[0]
    w[1440] = 4.0                # b3
    return SN.bf16_bits(w)


def compare(b, probs, **solo_kw):
    from paper_2007_14933_amd.batch import solo_run
    t_b, act, nact = b.status()
    assert nact == 0 and not act.any()
    for p, prob in enumerate(probs):
        s = solo_run(prob, cfl=b.cfl, **solo_kw)
        a, ref = b.state(p), s.state()
        same = np.array_equal(a, ref)
        say("   problem %d N=%d t=%.6g (solo %.6g, %d steps) bitwise %s max|diff| %.3e" % (
            p, prob.n[0], t_b[p], s.t, s.nsteps_done, same, np.abs(a - ref).max()))
        assert t_b[p] == s.t
        assert same


@pytest.mark.parametrize("form,scheme,sensor", [(0, I.TENO5, 0), (0, I.WENOZ5, 0), (1, I.TENO5, 0),
                                                 (1, I.TENO5, 1), (0, I.TENO5, 1)])
def test_batch_equals_solo(form, scheme, sensor):
    from paper_2007_14933_amd.batch import Batch
    probs = ensemble(SIZES, 11, T_ENDS, scheme)
    kw = dict(form=form, sensor=sensor)
    if sensor:
        kw.update(weights=jump_sensor_bits(), threshold=0.5)
    say("[gpu batch] form %d scheme %d sensor %d sizes %s" % (form, scheme, sensor, SIZES))
    b = Batch(probs, cfl=0.5, **kw)
    steps = b.run(poll=7)
    b.check()
    if sensor:
        sm, tot = b.solvers[0].sensor_stats()
        say("   problem 0 smooth fraction at its last refresh %.3f" % (sm / tot))
    say("   batch finished after %d steps" % steps)
    compare(b, probs, **kw)


# rows of 64 and more interfaces: the batched x sweep runs with lanes along
# x, and the first wave of every row of the batched y sweep loads ahead into
# LDS; the others march
ORACLE_SIZES = (64, 100, 40, 72)
ORACLE_T_ENDS = (0.02, 0.012, 0.03, 0.016)


@pytest.mark.parametrize("form,scheme", [(0, I.TENO5), (0, I.WENOZ5), (1, I.TENO5)])
def test_batch_against_oracle(form, scheme):
    """Every batched problem against the FP64 oracle run of the same problem
    to its own end time: plain FP64 at the run-parity bar (max normwise
    relative difference <= 1e-11), the precision form at the bounds of its
    oracle tests (relative L1 of density <= 1e-4, energy <= 3e-4)."""
    from oracle import oracle as O
    from parity_util import normwise_rel, oracle_run
    from paper_2007_14933_amd.batch import Batch
    probs = ensemble(ORACLE_SIZES, 21, ORACLE_T_ENDS, scheme)
    say("[gpu batch vs oracle] form %d scheme %d sizes %s" % (form, scheme, ORACLE_SIZES))
    b = Batch(probs, cfl=0.5, form=form)
    b.run(poll=5)
    b.check()
    t_b, act, nact = b.status()
    assert nact == 0
    for p, prob in enumerate(probs):
        Uo, to = oracle_run(prob, 10 ** 6, cfl=0.5, t_end=prob.t_end)
        a, ref = O.interior(prob, b.state(p)), O.interior(prob, Uo)
        if form == 0:
            err = normwise_rel(a, ref)
            say("   problem %d N=%d t=%.6g (oracle %.6g) normwise rel diff %s" % (p, prob.n[0], t_b[p], to, err))
            assert abs(t_b[p] - to) <= 1e-12 * to
            assert err.max() <= 1e-11, err
        else:
            l1 = [np.abs(a[c] - ref[c]).mean() / np.abs(ref[c]).mean() for c in (0, prob.nc - 1)]
            say("   problem %d N=%d t=%.6g (oracle %.6g) rel L1 rho %.3e rhoE %.3e" % (p, prob.n[0], t_b[p], to, *l1))
            assert abs(t_b[p] - to) <= 1e-4 * to
            assert l1[0] <= 1e-4 and l1[1] <= 3e-4, l1


def test_batch_tiles_and_direct_launches_do_not_change_results():
    from paper_2007_14933_amd.batch import Batch
    probs = ensemble(SIZES, 12, T_ENDS)
    say("[gpu batch] tiles")
    ref = Batch(probs, capture=True)
    ref.run()
    # x knob: runs per tile for the rows of >= 64 interfaces (1 and 64 are its
    # ends), the marching segment for the others
    for seg, capture in ((1, False), (8, True), (64, False), (1024, True)):
        b = Batch(probs, capture=False)
        b.set_tiles(np.full((len(probs), 2), seg))
        if capture:
            b.capture()
        b.run(poll=5)
        for p in range(len(probs)):
            assert np.array_equal(b.state(p), ref.state(p)), (seg, capture, p)
        say("   seg %d capture %s: bitwise equal" % (seg, capture))


def test_graph_replays_with_eager_work_between():
    """Replays of the captured graphs interleaved with unrelated eager work
    and synchronisations agree with direct launches after every step."""
    import torch
    from paper_2007_14933_amd.batch import Batch
    probs = ensemble((40, 24, 56), 13, (1.0, 1.0, 1.0))
    g = Batch(probs, capture=True)
    d = Batch(probs, capture=False)
    junk = torch.randn(1 << 20, device="cuda:0", dtype=torch.float64)
    for k in range(6):
        g.step()
        junk = torch.sqrt(junk * junk + 1.0)  # eager work on another stream
        float(junk.sum())
        d.step()
        torch.cuda.synchronize()
        for p in range(len(probs)):
            assert np.array_equal(g.state(p), d.state(p)), (k, p)
    say("[gpu batch] 6 graph replays equal direct launches")


def test_tuner_picks_valid_tiles_and_keeps_results(tmp_path, monkeypatch):
    from paper_2007_14933_amd.batch import Batch
    monkeypatch.setenv("OSBLI_TILE_CACHE", str(tmp_path / "tiles.json"))
    # 64 and 80: rows of >= 64 interfaces (lanes-along-x sweep, x knob =
    # runs per tile); 32, 48: marching x sweep (x knob = segment)
    probs = ensemble((64, 32, 80, 48), 14, (0.02, 0.02, 0.02, 0.02))
    ref = Batch(probs)
    ref.run()
    b = Batch(probs)
    chosen = b.tune(nsteps=2, log=say)
    assert set(chosen) == {(64, 64), (32, 32), (80, 80), (48, 48)}
    for (nx, ny), (sx, sy) in chosen.items():
        assert 1 <= sx <= (64 if nx + 1 >= 64 else nx) and 1 <= sy <= ny
    rep = b.tune_report
    say("[gpu batch] tuned %s, default %.3f ms, tuned %.3f ms, sweep workgroups %d"
        % (chosen, rep["default_ms_per_step"], rep["tuned_ms_per_step"], rep["sweep_blocks"]))
    assert rep["sweep_blocks"] in (0, 512, 1024, 2048, 4096, 8192)
    assert (tmp_path / "tiles.json").exists()
    b.run()
    for p in range(len(probs)):
        assert np.array_equal(b.state(p), ref.state(p))
    # second call reads the cache
    again = Batch(probs).tune(nsteps=2)
    assert again == chosen


def test_batch_rejects_unsupported_problems():
    from paper_2007_14933_amd import binding as B
    from paper_2007_14933_amd.batch import Batch
    with pytest.raises(B.OsbliError):
        Batch([I.riemann2d(32, 1), I.tgv(16)])            # 3D, viscous
    a, c = I.riemann2d(32, 1), I.riemann2d(32, 2).with_(gamma=1.3)
    with pytest.raises(B.OsbliError):
        Batch([a, c])                                     # physics differ
    with pytest.raises(B.OsbliError):
        Batch([I.riemann2d(32, 1)], t_end=[-1.0])         # bad end time
