"""Failure detection and restart on the production path.

* A run past the stability limit is caught by the propagator's periodic health check within K steps
  of its first non-finite level, on every schedule; a stable run is never flagged.
* Kill and resume: a forward run stopped after some step, its state (u^n, u^{n-1}) written to disk and
  read back into a new propagator, continues bitwise as if it had never stopped (fields and traces).
"""
import numpy as np
import pytest

from paper_1603_03971_amd import synth

pytestmark = pytest.mark.gpu


def _parse(schedule):
    """"sched[-ghosts[-halo]]" -> (sched, ghosts, halo), with "ring" and "region" by default."""
    parts = schedule.split("-")
    return parts[0], parts[1] if len(parts) > 1 else "ring", parts[2] if len(parts) > 2 else "region"


def _say(msg):
    print(msg, flush=True)


def _setup(n, fraction, schedule, check_every, nsteps=3000):
    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Propagator, Sources

    h, v = 10.0, 2000.0
    dt = Grid.stable_dt(4, h, v, fraction)
    g = Grid(n, n, n, h, dt, sponge_width=6)
    kap = g.kappa_from_velocity(synth.constant_velocity((n, n, n), v))
    c = n // 2
    src = Sources(g, [(c, c, c)], g.injection_weights([v]), g.ricker(nsteps, 15.0)[:, None])
    prop = Propagator(g, kap, sources=src, receivers=[(c, c, 4)], schedule=schedule, check_every=check_every)
    return g, prop


def _first_raise(prop, limit):
    for _ in range(limit):
        try:
            prop.step()
        except FloatingPointError as e:
            return prop.n, str(e)
    return None, None


@pytest.mark.parametrize("schedule", ["serial", "overlap", "fused"])
def test_unstable_run_is_caught_within_k_steps(schedule):
    """dt at 1.05 times the stability limit: the check with K = 1 finds the first non-finite level;
    with K = 16 the run raises at the first multiple of 16 at or after it."""
    n1, msg = _first_raise(_setup(40, 1.05, schedule, 1)[1], 3000)
    assert n1 is not None, "the unstable run never went non-finite"
    n16, _ = _first_raise(_setup(40, 1.05, schedule, 16)[1], 3000)
    _say(f"{schedule}: first non-finite level {n1} ({msg}); K = 16 raised at level {n16}")
    assert n16 == -(-n1 // 16) * 16
    assert n16 - n1 < 16


def test_stable_run_is_not_flagged():
    g, prop = _setup(40, 0.99, "serial", 10)
    for _ in range(800):
        prop.step()
    assert prop.n == 800


@pytest.mark.parametrize("schedule", ["serial", "fused", "serial-slots", "serial-slots-shell"])
def test_kill_and_resume_is_bitwise(tmp_path, schedule):
    """-slots: ghosts read from the receive slots; the resumed run primes them from the saved level.
    -shell: the shell form of the halo call, which also reads the faces of the two saved levels."""
    import torch

    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Propagator, Sources

    shape = (40, 36, 72)
    v = np.array(synth.layered_velocity(shape, 10.0, seed=12))
    h, nsteps, stop = 10.0, 90, 37
    dt = Grid.stable_dt(4, h, float(v.max()))
    g = Grid(shape[2], shape[1], shape[0], h, dt, sponge_width=8)
    kap = g.kappa_from_velocity(v)
    src_ijk = [(36, 18, 20), (2, 30, 5)]
    w = g.injection_weights([v[20, 18, 36], v[5, 30, 2]])
    amp = np.repeat(g.ricker(nsteps, 15.0)[:, None], 2, axis=1)
    rec = [(10, 10, 3), (70, 35, 39)]

    def fresh():
        sched, ghosts, halo = _parse(schedule)
        return Propagator(g, kap, sources=Sources(g, src_ijk, w, amp), receivers=rec, schedule=sched,
                          ghosts=ghosts, halo=halo)

    ref = fresh()
    tr_ref = ref.new_traces(nsteps)
    ref.run(nsteps, tr_ref)
    torch.cuda.synchronize()

    a = fresh()
    tr_a = a.new_traces(nsteps)
    a.run(stop, tr_a)
    torch.cuda.synchronize()
    path = tmp_path / "state.npz"
    np.savez(path, u_cur=g.download(a.u_cur), u_prv=g.download(a.u_prv), n=a.n, traces=tr_a.cpu().numpy())
    del a, tr_a                                     # the run is gone

    saved = np.load(path)
    b = fresh()
    b.set_state(saved["u_cur"], saved["u_prv"], n=int(saved["n"]))
    tr_b = torch.from_numpy(saved["traces"]).to(g.device)
    b.run(nsteps - stop, tr_b)
    torch.cuda.synchronize()
    assert b.n == nsteps
    assert np.array_equal(g.download(b.u_cur), g.download(ref.u_cur))
    assert np.array_equal(g.download(b.u_prv), g.download(ref.u_prv))
    assert torch.equal(tr_b, tr_ref)
