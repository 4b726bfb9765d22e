"""Checkpoint and resume: a run interrupted after three steps, saved,
restored into a fresh context and continued matches the uninterrupted run
bit for bit (fields everywhere, particles by id), in FP64 and in the mixed
form; a checkpoint is refused while injections are queued and by a context
of another configuration."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def case(precision):
    p = W.scaled(W.config("c2"), 16, 16, 32, n_e=4000, n_ion=4000, n_n=6000)
    p["collisions"] = dict(p["collisions"])
    p["collisions"].update(sigma_el=3e-17, lotz_a=4.5e-15)
    p["precision"] = precision
    return p


def make(p):
    from paper_2606_05893_amd import pic as G
    gpu = G.Pic(p, capacity=(40000, 40000, 40000))
    pre = W.preload(p, seed=21)
    for s, (pos, vel, ids) in pre.items():
        gpu.load(s, pos, vel, ids)
    gpu.set_clock(0, sum(v[0].shape[0] for v in pre.values()))
    return gpu


def state(gpu):
    out = {"fields": [a.cpu().numpy() for a in gpu.read_fields()]}
    for s in range(3):
        pos, vel, ids = (a.cpu().numpy() for a in gpu.read(s))
        o = np.argsort(ids)
        out[s] = (ids[o], pos[o], vel[o])
    return out


@pytest.mark.parametrize("warm", ["prev", "extrap"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resume_matches_uninterrupted_run(gpu_lib, precision, warm):
    """With the extrapolated start the checkpoint carries the potential of
    the solve before the last too, so the resumed run extrapolates from the
    same pair."""
    from paper_2606_05893_amd import pic as G
    p = case(precision)
    dt = p["dt"]
    a = make(p)
    a.set_warm_start(warm)
    da = [a.step(dt)[1] for _ in range(6)]
    b = make(p)
    b.set_warm_start(warm)
    for _ in range(3):
        b.step(dt)
    blob = b.checkpoint()
    del b
    c = G.Pic(p, capacity=(40000, 40000, 40000))
    c.set_warm_start(warm)
    c.restore(blob)
    dc = [c.step(dt)[1] for _ in range(3)]
    assert sum(d["ionisations"] for d in da) > 0
    for x, y in zip(da[3:], dc):
        for k in ("counts", "cathode", "anode", "ionisations", "elastic",
                  "candidates", "starved", "fn_emitted", "total_charge_units",
                  "step", "next_id"):
            assert x[k] == y[k], (k, x[k], y[k])
        assert x["solve"]["vcycles"] == y["solve"]["vcycles"]
        assert x["field_energy"] == y["field_energy"]
    sa, sc = state(a), state(c)
    for fa, fc in zip(sa["fields"], sc["fields"]):
        assert np.array_equal(fa, fc)
    for s in range(3):
        for xa, xc in zip(sa[s], sc[s]):
            assert np.array_equal(xa, xc), s


def test_checkpoint_refusals(gpu_lib):
    from paper_2606_05893_amd import pic as G
    p = case("fp64")
    a = make(p)
    a.step(p["dt"])
    pos, vel, _ = W.random_particles(10, p, 5, z_margin=1)
    a.inject(0, pos, vel)
    with pytest.raises(G.PicError):
        a.checkpoint()
    a.step(p["dt"])
    blob = a.checkpoint()
    q = W.scaled(W.config("c2"), 16, 16, 16, n_e=10, n_ion=10, n_n=10)
    other = G.Pic(q, capacity=(40000, 40000, 40000))
    with pytest.raises(G.PicError):
        other.restore(blob)
    with pytest.raises(G.PicError):
        G.Pic(p, capacity=(40000, 40000, 40000)).restore(blob[:100])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_step_matches_its_three_stages(gpu_lib, precision):
    """Six steps of pic_step give the same state, bit for bit, as six
    rounds of pic_deposit, pic_field and pic_advance (fields, particles by
    id, the per-step counts; kinetic energies to rounding), with queued
    injections of every species in between."""
    p = case(precision)
    dt = p["dt"]
    a, b = make(p), make(p)
    for k in range(6):
        for s in range(3):
            pos, vel, _ = W.random_particles(20, p, 300 + 10 * k + s, z_margin=1)
            a.inject(s, pos, vel)
            b.inject(s, pos, vel)
        _, da = a.step(dt)
        b.deposit()
        b.field()
        _, db = b.advance(dt)
        for key in ("counts", "cathode", "anode", "ionisations", "elastic",
                    "candidates", "starved", "fn_emitted", "total_charge_units",
                    "emitted", "step", "next_id"):
            assert da[key] == db[key], (k, key, da[key], db[key])
        # Kinetic energies are sums over workgroup partials, and the order
        # of particles inside a tile (hence the grouping) comes from atomics.
        assert np.allclose(da["kinetic"], db["kinetic"], rtol=1e-12, atol=0)
    assert sum(d for d in da["counts"]) > 0
    sa, sb = state(a), state(b)
    for fa, fb in zip(sa["fields"], sb["fields"]):
        assert np.array_equal(fa, fb)
    for s in range(3):
        for xa, xb in zip(sa[s], sb[s]):
            assert np.array_equal(xa, xb), s
