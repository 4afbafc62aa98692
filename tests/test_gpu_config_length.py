"""Parity at the lengths of the benchmark configurations (needs an MI355X).

* The plain binary64 lattice (64 x 128, 20 % filling, 0.5 V, Ea = 0.3 eV):
  all 10,000 steps in lockstep with the oracle, the near-threshold draws
  logged by both sides counted, and the tagged-ion mean squared displacement
  from snapshots every 100 steps (the j-th ion of a rail is its j-th occupied
  site: ions never pass each other), equal on both sides.
* The large device's tiling (1024-site rails, one-rail wave tiles, binary32,
  per-site barriers, the +-2 V sweep) on 128 rails: 2048 steps (two
  1024-step launches) in full lockstep.
* The large device itself (4096 x 1024) to 64 steps (a table window of the
  wave kernel): windows of rails checked through their light cone (the
  oracle updates 300 consecutive rails, the rails outside frozen; a frozen
  rail's error reaches one rail further per half-step, so the middle 44 rails
  are exact after 128 half-steps).
"""
import numpy as np
import pytest

import oracle
from parity_util import gpu_available, lockstep
from workloads import c1_plain_fp64, c2_large_device, gaussian_barriers, triangle

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _tagged_positions(occ, rails, sites):
    o = occ.reshape(rails, sites)
    return [np.nonzero(row)[0] for row in o]


def test_c1_all_steps_with_msd():
    from paper_2511_09413_amd import Simulator
    wl = c1_plain_fp64(n_steps=10_000)
    p_or = oracle.OracleParams(wl.physics, wl.rails, wl.sites)
    occ0 = oracle.fill(p_or, wl.filling)
    sim = Simulator(wl.physics, wl.rails, wl.sites)
    sim.load_occupancy(occ0)
    sim.set_protocols(wl.protocols)
    R, L = wl.rails[0], wl.sites[0]
    start = _tagged_positions(occ0, R, L)
    msd_gpu, msd_or = [], []
    occ_o = occ0.copy()
    logged = 0
    for k in range(100):
        st = lockstep(sim, p_or, wl.protocols, occ_o, 100, 100)
        assert st["resyncs"] == 0
        logged += st["oracle_log"]
        assert st["gpu_log"] == st["oracle_log"]
        occ_o = st["occ"]
        g = _tagged_positions(sim.read_occupancy(), R, L)
        o = _tagged_positions(occ_o, R, L)
        msd_gpu.append(np.mean(np.concatenate([(a - b) ** 2 for a, b in zip(g, start)])))
        msd_or.append(np.mean(np.concatenate([(a - b) ** 2 for a, b in zip(o, start)])))
    assert sim.step == 10_000
    assert msd_gpu == msd_or
    # the MSD grows from 0 over the run, of the order of 2 p t (p ~ 1e-5 per
    # attempt, two attempts per step): a fraction of a site squared
    assert 0.0 < msd_gpu[-1] < 2.0 and msd_gpu[-1] >= msd_gpu[9]
    print(f"c1 10000 steps: msd(t=1e4) = {msd_gpu[-1]:.4f} sites^2, near-threshold draws logged: {logged}")


def test_c2_tiling_2048_steps_lockstep():
    from paper_2511_09413_amd import Simulator
    wl = c2_large_device(n_steps=100_000)
    R, L = 128, 1024
    ea = gaussian_barriers((R, L), 0.3, 0.02, seed=2, dtype=np.float32)
    sim = Simulator(wl.physics, [R], [L], ea=ea)
    assert sim.launch_mode == "wave"
    p_or = oracle.OracleParams(wl.physics, [R], [L], ea)
    occ0 = oracle.fill(p_or, [0.3])
    sim.load_occupancy(occ0)
    protos = [triangle(2.0, 100_000 * wl.physics.dt_s)]
    sim.set_protocols(protos)
    st = lockstep(sim, p_or, protos, occ0, 2048, 1024)
    assert st["hops"] > 200
    print(f"c2 tiling 128x1024, 2048 steps: {st['hops']} hops, resyncs {st['resyncs']}, "
          f"near-threshold draws {st['oracle_log']}")


def test_c2_full_size_64_steps_light_cone():
    from paper_2511_09413_amd import Simulator
    wl = c2_large_device(n_steps=100_000)
    ea = wl.ea_site - np.float32(0.17)       # lower barriers: thousands of hops per step
    sim = Simulator(wl.physics, wl.rails, wl.sites, ea=ea)
    assert sim.launch_mode == "wave"
    sim.fill_random(wl.filling)
    occ0 = sim.read_occupancy()
    sim.set_protocols(wl.protocols)
    net, _ = sim.run_steps(64, tallies=True)
    occ = sim.read_occupancy().reshape(4096, 1024)
    assert (occ.sum(axis=1) == occ0.reshape(4096, 1024).sum(axis=1)).all()
    assert int(np.abs(net.cpu().numpy()).sum()) > 1000
    p_or = oracle.OracleParams(wl.physics, wl.rails, wl.sites, ea)
    oracle.set_threads(8)
    try:
        for lo in (0, 1900, 4096 - 300):
            part = occ0.copy()
            oracle.run(p_or, wl.protocols, part, 0, 64, rail_lo=lo, rail_hi=lo + 300, want_dec=False)
            ref = part.reshape(4096, 1024)
            assert np.array_equal(occ[lo + 128:lo + 172], ref[lo + 128:lo + 172]), lo
    finally:
        oracle.set_threads(1)
