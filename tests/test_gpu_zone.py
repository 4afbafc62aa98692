"""The paper's zone model on the GPU (kmc_zone_*) against the oracle's zone
model, step by step (needs an MI355X).

Both sides evaluate the table of Eqs. S1-S4 in binary64 from the same zone
populations and draw the same Philox uniforms, so trajectories, per-step net
moves and zone populations are identical (a decision could differ only if a
uniform, a multiple of 2^-32, fell between the two sides' values of one
probability, which differ at most in the last bit of exp)."""
import numpy as np
import pytest

import oracle
from parity_util import gpu_available
from workloads import constant, step_then_relax, triangle, zone_positions, zone_relaxation

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _occ(X, rails, sites):
    occ = np.zeros((rails, sites), dtype=np.int8)
    for i, row in enumerate(X):
        occ[i, row - 1] = 1
    return occ.reshape(-1)


def _pair(rails, sites, ions, zones, p0, vf, seed, kT=0.0258, dt=1e-3):
    from paper_2511_09413_amd import ZoneSimulator
    X0 = zone_positions(rails, sites, ions, seed + 1) if ions else np.zeros((rails, 0), dtype=np.int32)
    sim = ZoneSimulator(rails, sites, ions, zones=zones, p0=p0, kT_ev=kT, v_factor=vf, dt_s=dt, seed=seed,
                        occ=_occ(X0, rails, sites))
    p = oracle.ZoneParams(rails, ions, sites, zones=zones, p0=p0, kT=kT, v_factor=vf, dt=dt, seed=seed)
    return sim, p, X0.copy()


@pytest.mark.parametrize("rails,sites,ions,zones,p0,vf,proto", [
    (64, 200, 60, 10, 0.5, 5e-4, triangle(5.0, 0.3)),
    (7, 37, 13, 10, 0.9, 1e-2, step_then_relax(3.0, 0.02)),     # odd ions, zones of unequal width
    (3, 50, 1, 10, 0.7, 0.0, constant(-2.0)),                     # one ion per rail, odd rail count
    (5, 64, 64, 10, 0.8, 1e-3, constant(4.0)),                    # full rails: nothing can move
    (9, 130, 64, 7, 0.6, 2e-3, triangle(-6.0, 0.2)),              # 64 ions (every lane), 7 zones
    (4, 90, 63, 10, 0.95, 1e-3, constant(1.0)),                   # dense rails, last lane half used
    (33, 20, 0, 10, 0.5, 1e-3, constant(1.0)),                    # no ions
    (1, 2, 1, 1, 1.0, 0.0, constant(0.0)),                        # the smallest rail
])
def test_zone_trajectory_equals_oracle(rails, sites, ions, zones, p0, vf, proto):
    sim, p, X = _pair(rails, sites, ions, zones, p0, vf, seed=rails * 131 + sites)
    sim.set_bias_protocol(*proto)
    moved = 0
    for chunk in (1, 40, 160):
        net_g, zon_g = sim.run_steps(chunk, tallies=True)
        out = oracle.zone_run(p, proto, X, sim.step - chunk, chunk)
        assert np.array_equal(net_g.cpu().numpy(), out["net"])
        assert np.array_equal(zon_g.cpu().numpy(), out["zones"])
        assert np.array_equal(sim.read_positions(), X)
        assert np.array_equal(sim.read_occupancy(), _occ(X, rails, sites))
        moved += int(np.abs(out["net"]).sum())
    if 0 < ions < sites and p0 > 0:
        assert moved > 0


def test_zone_protocol_install_and_reload():
    """A protocol installed mid-run starts at the current step; a reloaded
    occupancy restarts from the new state."""
    sim, p, X = _pair(16, 100, 30, 10, 0.6, 3e-3, seed=77)
    sim.set_bias_protocol(*triangle(4.0, 0.1))
    sim.run_steps(50)
    oracle.zone_run(p, triangle(4.0, 0.1), X, 0, 50)
    proto2 = step_then_relax(-3.0, 0.03)
    sim.set_bias_protocol(*proto2)
    net_g, zon_g = sim.run_steps(80, tallies=True)
    out = oracle.zone_run(p, proto2, X, 50, 80, n_set=50)
    assert np.array_equal(net_g.cpu().numpy(), out["net"]) and np.array_equal(sim.read_positions(), X)
    X2 = zone_positions(16, 100, 30, 991)
    sim.load_occupancy(_occ(X2, 16, 100))
    net_g, _ = sim.run_steps(60, tallies=True)
    out = oracle.zone_run(p, proto2, X2, 130, 60, n_set=50)
    assert np.array_equal(net_g.cpu().numpy(), out["net"]) and np.array_equal(sim.read_positions(), X2)


def test_zone_rejects_unequal_rails():
    from paper_2511_09413_amd import KmcError, ZoneSimulator
    occ = np.zeros((2, 10), dtype=np.int8)
    occ[0, :3] = 1
    occ[1, :4] = 1
    with pytest.raises(KmcError):
        ZoneSimulator(2, 10, 3, occ=occ.reshape(-1))


def test_zone_table_s2_full_size():
    """128,000 rails x 200 columns, 60 ions per rail (Table S2's largest run,
    Table S1's constants): 6 steps of the polarising 5 V pulse, the whole
    lattice against the oracle (every rail couples to every other through the
    zone populations)."""
    wl = zone_relaxation(rails=128_000, n_steps=6)
    from paper_2511_09413_amd import ZoneSimulator
    sim = ZoneSimulator(wl.rails, wl.sites, wl.ions, zones=wl.zones, p0=wl.p0, kT_ev=wl.kT_ev,
                        v_factor=wl.v_factor, dt_s=wl.dt_s, seed=wl.seed, occ=wl.occupancy())
    sim.set_bias_protocol(*wl.protocol)
    net_g, zon_g = sim.run_steps(wl.n_steps, tallies=True)
    p = oracle.ZoneParams(wl.rails, wl.ions, wl.sites, zones=wl.zones, p0=wl.p0, kT=wl.kT_ev,
                          v_factor=wl.v_factor, dt=wl.dt_s, seed=wl.seed)
    X = wl.X0.copy()
    out = oracle.zone_run(p, wl.protocol, X, 0, wl.n_steps)
    assert np.array_equal(net_g.cpu().numpy(), out["net"])
    assert np.array_equal(zon_g.cpu().numpy(), out["zones"])
    assert np.array_equal(sim.read_positions(), X)
    assert np.abs(out["net"]).sum() > 100000
