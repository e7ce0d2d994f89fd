"""GPU parity: the HIP library through its C ABI against the FP64 oracle on
the same seeded inputs.  FP64 paths must agree per real component to 1e-12
(links) and 1e-13 (plaquettes); FP32 paths within the tolerances derived in
the design notes (storage rounding 6e-8 per component, amplified by the few
hundred operations of a sweep)."""
import os

import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1510_04675_amd as msmc
    msmc.lib()
    return msmc


@pytest.fixture(scope="module", autouse=True)
def _threads(orc):
    orc.set_threads(min(16, os.cpu_count() or 1))


def field(m, dims, prec="fp64"):
    return m.Field(dims, prec)


def P(n_or=4, hits=1, tries=64, reunit=0, sampler=0):
    import paper_1510_04675_amd as msmc
    return msmc.hb_params(n_or, hits, tries, reunit, sampler)


def test_hot_start_matches_oracle(m, orc):
    for d in ([4, 4, 4, 4], [6, 2, 4, 8]):
        f = field(m, d)
        m.su3_init_hot(f, 1, 3)
        U = m.su3_field_to_host(f)
        ref = orc.init_hot(d, 1, 3)
        assert np.max(np.abs(U - ref)) < 1e-14


def test_host_roundtrip_and_precisions(m, orc):
    d = [4, 6, 2, 4]
    U = si.random_field(d, 5)
    f = field(m, d)
    m.su3_field_from_host(f, U)
    assert np.array_equal(m.su3_field_to_host(f), U)
    g = field(m, d, "fp32")
    m.su3_field_from_host(g, U)
    assert np.array_equal(m.su3_field_to_host(g), U.astype(np.float32).astype(np.float64))
    r = field(m, d, "fp32_r12")
    m.su3_field_from_host(r, U)
    assert np.max(np.abs(m.su3_field_to_host(r) - U)) < 1e-6
    h = field(m, d)
    m.su3_field_copy(h, g)
    assert np.array_equal(m.su3_field_to_host(h), m.su3_field_to_host(g))


def test_plaquette_action_charge_energy_match_oracle(m, orc):
    d = [6, 4, 4, 6]
    U = si.random_field(d, 7)
    orc.wilson_flow(d, U, 0.05, 3)  # smoother field so Q is not pure noise
    f = field(m, d)
    m.su3_field_from_host(f, U)
    assert abs(m.su3_plaquette(f) - orc.plaquette(d, U)) < 1e-13
    assert abs(m.su3_action(f, 5.7) - orc.action(d, U, 5.7)) < 1e-9
    assert abs(m.su3_topological_charge(f) - orc.topological_charge(d, U)) < 1e-11
    assert abs(m.su3_clover_energy(f) - orc.clover_energy(d, U)) < 1e-12


@pytest.mark.parametrize("prec", ["fp32", "fp32_r12"])
def test_reduced_precision_plaquette_of_the_same_field(m, orc, prec):
    """Measurement parity: the plaquette of an FP32 / FP32-R12 field (R12
    uses the SU(3) row identity in fp32 per plaquette, summed in fp64)
    against the oracle's FP64 plaquette of exactly the stored links, to 1e-7;
    ragged extents and several blocks."""
    d = [10, 6, 4, 6]
    U = si.random_field(d, 12)
    orc.wilson_flow(d, U, 0.02, 2)
    f = field(m, d, prec)
    m.su3_field_from_host(f, U)
    Uh = m.su3_field_to_host(f)
    p = m.su3_plaquette(f)
    pref = orc.plaquette(d, Uh)
    print(f"{prec}: plaquette {p:.12f} oracle {pref:.12f}")
    assert abs(p - pref) < 1e-7


@pytest.mark.parametrize("prec", ["fp64", "fp32_r12"])
def test_wilson_loops_match_oracle(m, orc, prec):
    """m x n loops, partially averaged plaquettes (by chi_munu) and
    displaced 2 x 2 loops (by chi) against the oracle on the stored links of
    a smoothed ragged field; 1 x 1 equals the plaquette."""
    d = [6, 4, 8, 10]
    U = si.random_field(d, 21)
    orc.wilson_flow(d, U, 0.03, 4)
    f = field(m, d, prec)
    m.su3_field_from_host(f, U)
    Uh = m.su3_field_to_host(f)
    tol = 1e-13 if prec == "fp64" else 1e-7
    assert abs(m.su3_wilson_loop(f, 1, 1) - orc.plaquette(d, Uh)) < tol
    for a, b in ((1, 2), (2, 1), (2, 3), (3, 3)):
        assert abs(m.su3_wilson_loop(f, a, b) - orc.wilson_loop(d, Uh, a, b)) < tol, (a, b)
    pp = m.su3_partial_plaquettes(f)
    dl = m.su3_displaced_loops(f)
    for k in range(3):
        assert abs(pp[k] - orc.partial_plaquette(d, Uh, k)) < tol, k
    for k in range(5):
        assert abs(dl[k] - orc.displaced_2x2(d, Uh, k)) < tol, k
    # the class averages recombine to the full averages
    assert abs((pp[0] + 2 * pp[1] + pp[2]) / 4 - m.su3_wilson_loop(f, 1, 1)) < tol
    assert abs(np.dot([1, 4, 6, 4, 1], dl) / 16 - m.su3_wilson_loop(f, 2, 2)) < tol


def test_gauge_transform_matches_oracle(m, orc):
    d = [4, 4, 2, 4]
    U = si.random_field(d, 8)
    f = field(m, d)
    m.su3_field_from_host(f, U)
    m.su3_gauge_transform(f, 44)
    orc.gauge_transform(d, U, 44)
    assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 1e-13


def test_config1_fp64_ten_sweeps_per_link(m, orc):
    """4^4, beta = 6, FP64, hot start (seed 1), 10 sweeps of 1 HB + 4 OR:
    every real component of the final 1024 links within 1e-12 and all ten
    plaquettes within 1e-13 of the oracle."""
    d = [4, 4, 4, 4]
    f = field(m, d)
    m.su3_init_hot(f, 1, 0)
    h = m.su3_sweep_hb_or(f, 6.0, 1, 0, 0, 10, P())
    U = orc.init_hot(d, 1, 0)
    href, ex = orc.sweep_hb_or(d, U, 6.0, 1, 0, 0, 10)
    assert ex == 0 and m.su3_last_exhausted(f) == 0
    assert np.max(np.abs(h - href)) < 1e-13
    assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 1e-12


def test_fp64_ragged_lattice_several_blocks(m, orc):
    """12x10x6x8: 2880 links per phase = 11.25 blocks of 256 (ragged tail),
    non-power-of-two extents, reunitarization every 2 sweeps, first_sweep 7."""
    d = [12, 10, 6, 8]
    f = field(m, d)
    m.su3_init_hot(f, 9, 2)
    h = m.su3_sweep_hb_or(f, 5.8, 9, 2, 7, 3, P(n_or=2, reunit=2))
    U = orc.init_hot(d, 9, 2)
    href, _ = orc.sweep_hb_or(d, U, 5.8, 9, 2, 7, 3, n_or=2, reunit_every=2)
    assert np.max(np.abs(h - href)) < 1e-13
    assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 1e-12


@pytest.mark.parametrize("sampler,hits,tries", [(1, 1, 64), (0, 3, 64), (0, 1, 1), (1, 2, 1)])
def test_sampler_hits_and_exhaustion_match_oracle(m, orc, sampler, hits, tries):
    d = [4, 2, 4, 2]
    f = field(m, d)
    m.su3_init_hot(f, 4, 0)
    beta = 1.0 if tries == 1 else 6.0
    h = m.su3_sweep_hb_or(f, beta, 4, 0, 0, 3, P(n_or=1, hits=hits, tries=tries, sampler=sampler))
    U = orc.init_hot(d, 4, 0)
    href, ex = orc.sweep_hb_or(d, U, beta, 4, 0, 0, 3, n_or=1, n_hb_hits=hits, hb_max_tries=tries, sampler=sampler)
    assert m.su3_last_exhausted(f) == ex
    if tries == 1:
        assert ex > 0
    assert np.max(np.abs(h - href)) < 1e-13
    assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 1e-12


@pytest.mark.parametrize("gbytes", [224 << 20, 1])
def test_batch_exhaustion_counts_per_lattice(m, orc, gbytes):
    """With one heat-bath trial per draw at beta = 1 many draws are left
    unchanged; after a batched call each field reports its own lattice's
    count (equal to the oracle's for that lattice alone), whether the batch
    runs as one lattice group or one group per lattice, and 0 after a call
    of no sweeps."""
    shapes = [[4, 4, 4, 4], [4, 2, 4, 2], [6, 4, 2, 4]]
    betas = [1.0, 0.8, 1.2]
    m.su3_set_group_bytes(gbytes)
    try:
        fs = [field(m, d) for d in shapes]
        for i, f in enumerate(fs):
            m.su3_init_hot(f, 30 + i, i)
        m.su3_batch_sweep_hb_or(fs, betas, [30, 31, 32], [0, 1, 2], 5, 2, P(n_or=1, tries=1))
        counts = [m.su3_last_exhausted(f) for f in fs]
    finally:
        m.su3_set_group_bytes(224 << 20)
    for i, d in enumerate(shapes):
        U = orc.init_hot(d, 30 + i, i)
        _, ex = orc.sweep_hb_or(d, U, betas[i], 30 + i, i, 5, 2, n_or=1, hb_max_tries=1)
        assert ex > 0
        assert counts[i] == ex, (i, counts, ex)
        assert np.max(np.abs(m.su3_field_to_host(fs[i]) - U)) < 1e-12
    # a call of no sweeps reports no exhausted draws, batched or not
    m.su3_batch_sweep_hb_or(fs[:2], betas[:2], [30, 31], [0, 1], 7, 0, P(n_or=1, tries=1))
    m.su3_sweep_hb_or(fs[2], betas[2], 32, 2, 7, 0, P(n_or=1, tries=1))
    assert [m.su3_last_exhausted(f) for f in fs] == [0, 0, 0]


@pytest.mark.parametrize("prec", ["fp64", "fp32_r12"])
def test_beta_zero_heat_bath_matches_oracle(m, orc, prec):
    """beta = 0, heat bath only: every draw exhausted on both sides (3 per
    link and hit), the fp64 links unchanged bit for bit and the 12-real
    plaquette unchanged to its rounding."""
    d = [4, 2, 4, 6]
    U = orc.init_hot(d, 6, 0)
    f = field(m, d, prec)
    m.su3_field_from_host(f, U)
    before = m.su3_field_to_host(f)
    p0 = m.su3_plaquette(f)
    m.su3_sweep_hb_or(f, 0.0, 6, 0, 0, 2, P(n_or=0, tries=3), record=False)
    _, ex = orc.sweep_hb_or(d, U, 0.0, 6, 0, 0, 2, n_or=0, hb_max_tries=3)
    assert ex == 2 * 3 * 4 * int(np.prod(d))
    assert m.su3_last_exhausted(f) == ex
    if prec == "fp64":
        assert np.array_equal(m.su3_field_to_host(f), before)
    else:
        assert abs(m.su3_plaquette(f) - p0) < 1e-6


def fp32_link_stats(Ugpu, Uref):
    """Per-link largest component deviation: median, 99.9th percentile, max."""
    dev = np.max(np.abs(Ugpu - Uref), axis=(2, 3, 4)).ravel()
    return float(np.median(dev)), float(np.quantile(dev, 0.999)), float(dev.max()), dev


@pytest.mark.parametrize("prec", ["fp32", "fp32_r12"])
def test_fp32_sweeps_track_fp64_oracle(m, orc, prec):
    """FP32 storage and arithmetic from the FP32-rounded copy of an
    oracle-thermalized field, one sweep of 1 HB + 1 OR (overrelaxation
    amplifies a perturbation about 5x per pass, so longer FP32 chains
    separate from the FP64 one by chaos, not by error).  Bars: plaquette
    within 1e-6 of the FP64 oracle; per-link deviation median below 1e-5 and
    99.9th percentile below 1e-3 (FP32 rounding 6e-8 amplified by the sweep;
    a flipped FP32 sampler decision would give an O(1) outlier, allowed for
    at most 1 link in 10^4)."""
    d = [8, 4, 4, 8]
    U = orc.init_hot(d, 2, 0)
    orc.sweep_hb_or(d, U, 6.0, 2, 0, 0, 8)
    f = field(m, d, prec)
    m.su3_field_from_host(f, U)
    h = m.su3_sweep_hb_or(f, 6.0, 2, 0, 100, 1, P(n_or=1, reunit=1))
    href, _ = orc.sweep_hb_or(d, U, 6.0, 2, 0, 100, 1, n_or=1, reunit_every=1)
    med, q999, mx, dev = fp32_link_stats(m.su3_field_to_host(f), U)
    print(f"{prec}: plaquette diff {abs(h[0] - href[0]):.2e}, link dev median {med:.2e} q99.9 {q999:.2e} max {mx:.2e}")
    assert abs(h[0] - href[0]) < 1e-6
    assert med < 1e-5 and q999 < 1e-3
    assert np.count_nonzero(dev > 1e-2) <= dev.size // 10000


def test_launch_shape_and_resume_invariance(m, orc):
    """Bitwise identical results for every launch shape (phase kernels, and
    the link walks of an HMC trajectory and of a flow), and N sweeps equal
    N/2 + N/2 sweeps."""
    d = [8, 6, 4, 4]
    ref = None
    shapes = [(64, 0, (0, 0, 1)), (128, 1, (2, 2, 2)), (256, 1, (3, 4, 4)), (512, 0, (6, 2, 1)), (512, 1, (16, 8, 4)),
              (256, 0, (1, 1, 4))]
    try:
        for block, remap, tile in shapes:
            m.su3_set_launch(block, remap)
            m.su3_set_tile(*tile)
            f = field(m, d, "fp32")
            m.su3_init_hot(f, 6, 1)
            m.su3_sweep_hb_or(f, 6.0, 6, 1, 0, 2, P(n_or=2))
            m.su3_sweep_hb_or(f, 6.0, 6, 1, 2, 2, P(n_or=2))
            U = m.su3_field_to_host(f)
            h = field(m, d, "fp32_r12")
            m.su3_field_copy(h, f)
            _, dh = m.su3_hmc_trajectory(h, 6.0, 1.0, 6, 6, 1, 3, 0)
            m.su3_wilson_flow(h, 0.02, 3)
            H = (dh, m.su3_field_to_host(h))
            if ref is None:
                ref, href = U, H
            assert np.array_equal(U, ref), (block, remap, tile)
            assert H[0] == href[0] and np.array_equal(H[1], href[1]), (block, remap, tile)
    finally:
        m.su3_set_launch(0, 1)
        m.su3_set_tile(0, 0, 0)
    f = field(m, d, "fp32")
    m.su3_init_hot(f, 6, 1)
    m.su3_sweep_hb_or(f, 6.0, 6, 1, 0, 4, P(n_or=2))
    assert np.array_equal(m.su3_field_to_host(f), ref)


def test_autotuned_shape_is_a_candidate_and_changes_nothing(m, orc):
    """The first sweep call on a new shape with the autotuner on picks one of
    the candidate launch shapes (block 128/256/512, remap 0/1, one of seven
    tiles) for that shape and leaves the results bitwise those of the default
    shape; the oracle agrees on the FP64 field."""
    d = [6, 8, 4, 4]
    U0 = orc.init_hot(d, 21, 0)
    res = {}
    try:
        for tuned in (False, True):
            m.su3_autotune(tuned)
            f = field(m, d)
            m.su3_field_from_host(f, U0)
            m.su3_sweep_hb_or(f, 6.0, 21, 0, 0, 2, P(n_or=2))
            res[tuned] = (m.su3_field_to_host(f), m.su3_get_config([f]))
    finally:
        m.su3_autotune(False)
    cfg = res[True][1]
    assert cfg["block"] in (128, 256, 512) and cfg["xcd_remap"] in (0, 1), cfg
    assert np.array_equal(res[True][0], res[False][0])
    U = U0.copy()
    orc.sweep_hb_or(d, U, 6.0, 21, 0, 0, 2, n_or=2)
    assert np.max(np.abs(res[True][0] - U)) < 1e-12


def test_batch_equals_separate_calls(m, orc):
    """One batched graph launch over lattices of uneven shapes gives bitwise
    the fields and plaquettes of separate calls, for any grouping of the
    lattices in the sweep schedule; replaying the cached graph continues the
    chain."""
    shapes = [[4, 4, 4, 4], [6, 4, 2, 4], [8, 2, 4, 6]]
    betas = [5.9, 6.05, 6.2]
    # group budget: one group, one lattice per group, the first two together
    budgets = [224 << 20, 1, 2 * 4 * 256 * 144 + 4 * 192 * 144]
    for prec, gbytes in (("fp64", budgets[0]), ("fp32_r12", budgets[0]), ("fp64", budgets[1]),
                         ("fp32_r12", budgets[1]), ("fp64", budgets[2])):
        m.su3_set_group_bytes(gbytes)
        fs = [field(m, d, prec) for d in shapes]
        gs = [field(m, d, prec) for d in shapes]
        for i, (a, b) in enumerate(zip(fs, gs)):
            m.su3_init_hot(a, 10 + i, i)
            m.su3_init_hot(b, 10 + i, i)
        for rep in range(2):
            pb = m.su3_batch_sweep_hb_or(fs, betas, [10, 11, 12], [0, 1, 2], 3 * rep, 3, P(n_or=2, reunit=2))
            for i, g in enumerate(gs):
                h = m.su3_sweep_hb_or(g, betas[i], 10 + i, i, 3 * rep, 3, P(n_or=2, reunit=2))
                assert np.array_equal(h, pb[:, i])
        for a, b in zip(fs, gs):
            assert np.array_equal(m.su3_field_to_host(a), m.su3_field_to_host(b))
    m.su3_set_group_bytes(224 << 20)
    # and the FP64 member matches the oracle
    d = shapes[1]
    U = orc.init_hot(d, 11, 1)
    orc.sweep_hb_or(d, U, 6.05, 11, 1, 0, 6, n_or=2, reunit_every=2)
    f = field(m, d)
    m.su3_init_hot(f, 11, 1)
    m.su3_batch_sweep_hb_or([f], [6.05], [11], [1], 0, 6, P(n_or=2, reunit=2))
    assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 1e-12


def test_hmc_trajectory_matches_oracle(m, orc):
    """FP64 HMC: momenta, leapfrog, dH and the Metropolis decision."""
    d = [4, 4, 4, 4]
    U = orc.init_hot(d, 5, 0)
    orc.sweep_hb_or(d, U, 6.0, 5, 0, 0, 5)
    f = field(m, d)
    m.su3_field_from_host(f, U)
    for traj in range(3):
        acc, dH = m.su3_hmc_trajectory(f, 6.0, 1.0, 12, 5, 0, traj, 1)
        racc, rdH = orc.hmc_trajectory(d, U, 6.0, 1.0, 12, 5, 0, traj, 1)
        assert acc == racc
        assert abs(dH - rdH) < 1e-8 * max(1.0, abs(rdH)), (dH, rdH)
        assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 1e-11
    # a rejected trajectory leaves the field unchanged bit for bit
    before = m.su3_field_to_host(f)
    acc, dH = m.su3_hmc_trajectory(f, 6.0, 4.0, 2, 5, 0, 99, 1)
    assert not acc and dH > 20
    assert np.array_equal(m.su3_field_to_host(f), before)


def test_hmc_coarse_steps_match_oracle(m, orc):
    """FP64 HMC with steps of 1/2: the drift's generators have norms near 1,
    beyond the 1/4 up to which the link exponential takes its polynomial
    directly, so it scales and squares.  Links and dH against the oracle's
    series summed to convergence (no Metropolis step, so the evolved field
    is kept)."""
    d = [4, 4, 4, 4]
    U = orc.init_hot(d, 8, 0)
    orc.sweep_hb_or(d, U, 6.0, 8, 0, 0, 4)
    f = field(m, d)
    m.su3_field_from_host(f, U)
    _, dH = m.su3_hmc_trajectory(f, 6.0, 1.0, 2, 8, 0, 4, 0)
    _, rdH = orc.hmc_trajectory(d, U, 6.0, 1.0, 2, 8, 0, 4, 0)
    assert abs(dH) > 1.0  # a coarse step: far from energy conservation
    assert abs(dH - rdH) < 1e-8 * max(1.0, abs(rdH)), (dH, rdH)
    assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 1e-11


def test_hmc_fp32_dh_tracks_fp64(m, orc):
    d = [8, 8, 4, 4]
    U = orc.init_hot(d, 6, 0)
    orc.sweep_hb_or(d, U, 6.0, 6, 0, 0, 5)
    f = field(m, d, "fp32")
    m.su3_field_from_host(f, U)
    acc, dH = m.su3_hmc_trajectory(f, 6.0, 1.0, 20, 6, 0, 0, 0)
    racc, rdH = orc.hmc_trajectory(d, U, 6.0, 1.0, 20, 6, 0, 0, 0)
    assert abs(dH - rdH) < 0.05 + 0.02 * abs(rdH), (dH, rdH)
    assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 5e-4


@pytest.mark.parametrize("prec", ["fp32", "fp32_r12"])
def test_hmc_reduced_precision_on_partial_rows(m, orc, prec):
    """The fp32 HMC step takes both parities of 64 positions per block and
    serves the +-x neighbours from the block's own links when they are there:
    on 6 x 4 x 8 x 6 an x row holds 3 positions, so blocks start and end in
    the middle of rows and some +-x neighbours belong to the next block.  One
    20-step trajectory against the oracle's from the same links."""
    d = [6, 4, 8, 6]
    U = orc.init_hot(d, 23, 0)
    orc.sweep_hb_or(d, U, 6.0, 23, 0, 0, 5)
    f = field(m, d, prec)
    m.su3_field_from_host(f, U)
    Uh = m.su3_field_to_host(f)
    _, dH = m.su3_hmc_trajectory(f, 6.0, 1.0, 20, 23, 0, 3, 0)
    _, rdH = orc.hmc_trajectory(d, Uh, 6.0, 1.0, 20, 23, 0, 3, 0)
    assert abs(dH - rdH) < 0.05 + 0.02 * abs(rdH), (dH, rdH)
    assert np.max(np.abs(m.su3_field_to_host(f) - Uh)) < 5e-4


@pytest.mark.parametrize("prec", ["fp32", "fp32_r12"])
def test_hmc_reduced_precision_dh_at_16_4(m, prec):
    """One 40-step trajectory on a thermalized 16^4 lattice in reduced
    precision against fp64 from the same links (fp64 is pinned to the oracle
    by the tests above).  dH is a difference of actions summed over 393216
    links, so a per-link bias of a fraction of an fp32 ulp in the stored links
    shows up here (an fp32 Gram-Schmidt in the 12-real drift gave 0.85 against
    0.61); rounding noise alone stays near 0.01."""
    d = [16] * 4
    f = field(m, d, prec)
    m.su3_init_cold(f)
    m.su3_sweep_hb_or(f, 6.0, 5, 0, 0, 30, m.hb_params(n_or=4, reunit_every=10), record=False)
    g = field(m, d, "fp64")
    m.su3_field_copy(g, f)
    _, dh = m.su3_hmc_trajectory(f, 6.0, 1.0, 40, 5, 0, 7, 0)
    _, dh64 = m.su3_hmc_trajectory(g, 6.0, 1.0, 40, 5, 0, 7, 0)
    h = field(m, d, "fp64")
    m.su3_field_copy(h, f)
    p_end, p64_end = m.su3_plaquette(f), m.su3_plaquette(h)
    print(f"\n{prec} 16^4 dH {dh:.5f} vs fp64 {dh64:.5f}; end plaquette {p_end:.10f} vs its fp64 copy {p64_end:.10f}")
    assert abs(dh - dh64) < 0.05, (dh, dh64)
    assert abs(p_end - p64_end) < 5e-9, (p_end, p64_end)


@pytest.mark.parametrize("prec", ["fp32", "fp32_r12"])
def test_hmc_reduced_precision_long_trajectory_at_32_4(m, prec):
    """A unit trajectory of 200 leapfrog steps (the step counts App. A needs
    on its finer lattices) at 32^4 from thermalized links, against fp64 from
    the same links: |dH - dH_fp64| < 0.05 and the stored links within 1e-6 of
    SU(3).  Every drift rounds the link update; without re-orthonormalizing
    the stored links those roundings carry the field away from SU(3) (1e-5
    after 240 steps) and dH off by an amount that grows faster than the step
    count (+0.5 after 182 steps at 32^3 x 72), which bent the acceptance
    curve of the finest App. A ensemble."""
    d = [32] * 4
    f = field(m, d, prec)
    m.su3_init_cold(f)
    m.su3_sweep_hb_or(f, 6.0, 5, 0, 0, 40, m.hb_params(n_or=4, reunit_every=10), record=False)
    g = field(m, d, "fp64")
    m.su3_field_copy(g, f)
    _, dh = m.su3_hmc_trajectory(f, 6.0, 1.0, 200, 5, 0, 11, 0)
    _, dh64 = m.su3_hmc_trajectory(g, 6.0, 1.0, 200, 5, 0, 11, 0)
    ok, dev, _ = m.su3_check_field(f, 1e-6)
    print(f"\n{prec} 32^4, 200 steps: dH {dh:.5f} vs fp64 {dh64:.5f}; largest deviation from SU(3) {dev:.2e}")
    assert abs(dh - dh64) < 0.05, (dh, dh64)
    assert ok and dev < 1e-6, dev


def test_wilson_flow_matches_oracle(m, orc):
    d = [4, 4, 6, 4]
    U = orc.init_hot(d, 3, 0)
    orc.sweep_hb_or(d, U, 6.0, 3, 0, 0, 3)
    f = field(m, d)
    m.su3_field_from_host(f, U)
    m.su3_wilson_flow(f, 0.02, 5)
    orc.wilson_flow(d, U, 0.02, 5)
    assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 1e-12
    assert abs(m.su3_topological_charge(f) - orc.topological_charge(d, U)) < 1e-11


def test_zero_length_trajectory_and_flow_are_identities(m, orc):
    """FP64 HMC with tau = 0 and flow steps of 0: the exponential of a zero
    generator is the identity and every kick zero, so the links come back bit
    for bit and dH is 0 exactly, as in the oracle."""
    d = [4, 2, 4, 6]
    U = orc.init_hot(d, 10, 0)
    f = field(m, d)
    m.su3_field_from_host(f, U)
    acc, dH = m.su3_hmc_trajectory(f, 6.0, 0.0, 5, 10, 0, 0, 1)
    assert acc and dH == 0.0
    assert np.array_equal(m.su3_field_to_host(f), U)
    m.su3_wilson_flow(f, 0.0, 3)
    assert np.array_equal(m.su3_field_to_host(f), U)


def test_coarse_flow_steps_match_oracle(m, orc):
    """FP64 flow steps of 0.5 from a hot start: stage generators beyond norm
    1/4, so the link exponential scales and squares; links and Q against the
    oracle."""
    d = [4, 4, 4, 6]
    U = orc.init_hot(d, 13, 0)
    f = field(m, d)
    m.su3_field_from_host(f, U)
    m.su3_wilson_flow(f, 0.5, 2)
    orc.wilson_flow(d, U, 0.5, 2)
    assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 1e-12
    assert abs(m.su3_topological_charge(f) - orc.topological_charge(d, U)) < 1e-11


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_r12"])
def test_adaptive_flow_matches_oracle(m, orc, prec):
    """Adaptive-step flow (tolerance 0.01, maximum step 0.2, first step 0.2
    so that rejections occur): FP64 takes the oracle's accepted and rejected
    steps and matches E, Q at the measurement times and the final links;
    FP32 and R12 match E to 1e-6 relative.  Admissibility h and the t0
    interpolation against the oracle on the same data."""
    d = [6, 4, 8, 6]
    U = orc.init_hot(d, 17, 0)
    orc.sweep_hb_or(d, U, 5.9, 17, 0, 0, 6)
    f = field(m, d, prec)
    m.su3_field_from_host(f, U)
    Uh = m.su3_field_to_host(f)
    tm = [0.0, 0.2, 0.4, 0.6, 0.9, 1.2]
    E, Q, na, nr = m.su3_wilson_flow_adaptive(f, 1.2, 0.01, 0.2, 0.2, tm)
    Er, Qr, nar, nrr = orc.wilson_flow_adaptive(d, Uh, 1.2, 0.01, 0.2, 0.2, tm)
    print(f"{prec}: steps {na}+{nr} rejected (oracle {nar}+{nrr}), E {E} oracle {Er}")
    assert nrr >= 1
    if prec == "fp64":
        assert (na, nr) == (nar, nrr)
        assert np.max(np.abs(E - Er)) < 1e-12 and np.max(np.abs(Q - Qr)) < 1e-11
        assert np.max(np.abs(m.su3_field_to_host(f) - Uh)) < 1e-11
        assert abs(m.su3_max_plaquette_action(f) - orc.max_splaq(d, Uh)) < 1e-12
    else:
        assert np.max(np.abs(E - Er) / Er) < 1e-6, np.abs(E - Er) / Er
        assert abs(m.su3_max_plaquette_action(f) - orc.max_splaq(d, m.su3_field_to_host(f))) < 1e-6
    tt = np.linspace(0.1, 2.0, 20)
    EE = (0.05 + 0.2 * tt) / tt**2  # t^2 E crosses 0.3 at t = 1.25
    assert abs(m.su3_flow_t0(tt, EE, 0.3) - orc.flow_t0(tt, EE, 0.3)) < 1e-15


@pytest.mark.parametrize("dc", [[2, 4, 2, 2], [4, 2, 6, 2]])
def test_restrict_and_prolongate_match_oracle(m, orc, dc):
    df = [2 * x for x in dc]
    Uc = orc.init_hot(dc, 7, 0)
    orc.sweep_hb_or(dc, Uc, 5.8, 7, 0, 0, 10)
    c = field(m, dc)
    fine = field(m, df)
    m.su3_field_from_host(c, Uc)
    it = m.su3_prolongate(c, fine, 0.05, 1e-5, 10000)
    Uf, rit = orc.prolongate(dc, Uc, 0.05, 1e-5, 10000)
    assert it == rit
    assert np.max(np.abs(m.su3_field_to_host(fine) - Uf)) < 1e-11
    c2 = field(m, dc)
    m.su3_restrict(fine, c2)
    assert np.max(np.abs(m.su3_field_to_host(c2) - orc.restrict(df, Uf))) < 1e-14
    assert np.max(np.abs(m.su3_field_to_host(c2) - Uc)) < 1e-14


@pytest.mark.parametrize("rel_tol,max_iter", [(1e-5, 1), (1e-5, 3), (0.0, 17), (1e-5, 0)])
def test_prolongate_step_caps_match_oracle(m, orc, rel_tol, max_iter):
    """Stopping by the step cap (1, 3, and 17: past a run of 16 enqueued steps),
    a tolerance that never stops early, and no steps at all: step counts and
    links as the oracle's."""
    dc = [2, 2, 4, 2]
    df = [2 * x for x in dc]
    Uc = orc.init_hot(dc, 5, 0)
    orc.sweep_hb_or(dc, Uc, 5.8, 5, 0, 0, 4)
    c = field(m, dc)
    fine = field(m, df)
    m.su3_field_from_host(c, Uc)
    it = m.su3_prolongate(c, fine, 0.05, rel_tol, max_iter)
    Uf, rit = orc.prolongate(dc, Uc, 0.05, rel_tol, max_iter)
    assert list(it) == list(rit)
    assert all(k <= max_iter for k in it)
    assert np.max(np.abs(m.su3_field_to_host(fine) - Uf)) < 1e-11


def test_check_field_flags_bad_links(m, orc):
    d = [4, 4, 4, 4]
    U = orc.init_hot(d, 1, 0)
    f = field(m, d)
    m.su3_field_from_host(f, U)
    ok, dev, _ = m.su3_check_field(f, 1e-12)
    assert ok and dev < 1e-14
    U[37, 2, 1, 1, 0] = np.nan
    m.su3_field_from_host(f, U)
    ok, dev, worst = m.su3_check_field(f, 1e-12)
    # site 37 has parity (1+1+2+0)%2 = 0, cb = 18, slab = 2*2+0
    assert not ok and worst == 4 * (np.prod(d) // 2) + 37 // 2


def test_full_size_32_4_fp64_sweep_matches_oracle(m, orc):
    """32^4 in the benchmark's launch shapes: one sweep (1 HB + 1 OR) from a
    hot start, every link compared with the oracle."""
    d = [32, 32, 32, 32]
    f = field(m, d)
    m.su3_init_hot(f, 3, 0)
    h = m.su3_sweep_hb_or(f, 6.0, 3, 0, 0, 1, P(n_or=1))
    U = orc.init_hot(d, 3, 0)
    href, _ = orc.sweep_hb_or(d, U, 6.0, 3, 0, 0, 1, n_or=1)
    assert abs(h[0] - href[0]) < 1e-13
    assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 1e-12


def test_full_size_32_4_fp32_sweep_tracks_oracle(m, orc):
    """32^4 FP32-R12, one sweep of 1 HB + 1 OR from the FP32-rounded copy of
    an oracle field (cold start + 3 sweeps at beta = 6): plaquette within
    1e-6 of the FP64 oracle; per-link deviation median below 1e-5, 99.9th
    percentile below 1e-3 and O(1) outliers (flipped FP32 sampler decisions)
    in at most 1 link in 10^4.  (From a Haar-random start the rough field
    amplifies FP32 rounding far more and only the plaquette bar applies.)"""
    d = [32, 32, 32, 32]
    U = orc.init_cold(d)
    orc.sweep_hb_or(d, U, 6.0, 3, 0, 0, 3, n_or=1)
    f = field(m, d, "fp32_r12")
    m.su3_field_from_host(f, U)
    h = m.su3_sweep_hb_or(f, 6.0, 3, 0, 3, 1, P(n_or=1))
    href, _ = orc.sweep_hb_or(d, U, 6.0, 3, 0, 3, 1, n_or=1)
    med, q999, mx, dev = fp32_link_stats(m.su3_field_to_host(f), U)
    print(f"32^4 r12: plaquette diff {abs(h[0] - href[0]):.2e}, link dev median {med:.2e} q99.9 {q999:.2e} max {mx:.2e}")
    assert abs(h[0] - href[0]) < 1e-6
    assert med < 1e-5 and q999 < 1e-3
    assert np.count_nonzero(dev > 1e-2) <= dev.size // 10000


def test_full_size_benchmark_batch_matches_oracle(m, orc):
    """The benchmark's workload at full size and in its launch configuration:
    4 x 32^4 R12 lattices (Haar hot starts, seed 3, lattice ids 0..3) swept
    as one batch with the autotuner on (lattice groups of at most 224 MiB,
    one lattice each), 1 HB + 4 OR passes at beta 6.  The first-sweep
    plaquette of lattices 0 and 3 lies within 1e-6 of the FP64 oracle's sweep
    of the same stored links (from the rough Haar start the chains separate
    per link by chaos within the sweep, so only the plaquette bar applies),
    and lattice 3 equals a separate call bitwise."""
    d = [32, 32, 32, 32]
    fs = [field(m, d, "fp32_r12") for _ in range(4)]
    for i, f in enumerate(fs):
        m.su3_init_hot(f, 3, i)
    starts = {i: m.su3_field_to_host(fs[i]) for i in (0, 3)}
    try:
        m.su3_autotune(True)
        pb = m.su3_batch_sweep_hb_or(fs, [6.0] * 4, [3] * 4, [0, 1, 2, 3], 0, 1, P(n_or=4, reunit=10))
    finally:
        m.su3_autotune(False)
    end3 = m.su3_field_to_host(fs[3])
    for f in fs[:3]:
        f.close()
    for i, U in starts.items():
        href, _ = orc.sweep_hb_or(d, U, 6.0, 3, i, 0, 1, n_or=4, reunit_every=10)
        print(f"\nlattice {i}: plaquette {pb[0, i]:.10f} oracle {href[0]:.10f}")
        assert abs(pb[0, i] - href[0]) < 1e-6
    g = field(m, d, "fp32_r12")
    m.su3_init_hot(g, 3, 3)
    h = m.su3_sweep_hb_or(g, 6.0, 3, 3, 0, 1, P(n_or=4, reunit=10))
    assert h[0] == pb[0, 3]
    assert np.array_equal(m.su3_field_to_host(g), end3)


def test_full_size_32_4_flow_steps_match_oracle(m, orc):
    """The Wilson flow at the benchmark's 32^4 and launch shapes (FP64: one
    link per thread; R12: the paired LDS walk): two RK3 steps of eps 0.02
    from the links of an R12 field roughened by one oracle sweep from a cold
    start.  FP64 per link within 1e-12 of the oracle's flow of the same
    links, plaquette 1e-12 and Q 1e-9; R12 plaquette within 2e-8 and Q within
    1e-4 (the bars of the 16^4 configuration)."""
    d = [32, 32, 32, 32]
    U = orc.init_cold(d)
    orc.sweep_hb_or(d, U, 6.0, 9, 0, 0, 1, n_or=1)
    fr = field(m, d, "fp32_r12")
    m.su3_field_from_host(fr, U)
    Ur = m.su3_field_to_host(fr)
    f64 = field(m, d, "fp64")
    m.su3_field_from_host(f64, Ur)
    m.su3_wilson_flow(f64, 0.02, 2)
    m.su3_wilson_flow(fr, 0.02, 2)
    p64, q64 = m.su3_plaquette(f64), m.su3_topological_charge(f64)
    pr, qr = m.su3_plaquette(fr), m.su3_topological_charge(fr)
    orc.wilson_flow(d, Ur, 0.02, 2)
    p_ref, q_ref = orc.plaquette(d, Ur), orc.topological_charge(d, Ur)
    d64 = float(np.max(np.abs(m.su3_field_to_host(f64) - Ur)))
    print(f"\n32^4 flow: P fp64 {p64:.12f} r12 {pr:.12f} oracle {p_ref:.12f}; Q fp64 {q64:.9f} r12 {qr:.9f} "
          f"oracle {q_ref:.9f}; fp64 max link diff {d64:.1e}")
    assert d64 < 1e-12
    assert abs(p64 - p_ref) < 1e-12 and abs(q64 - q_ref) < 1e-9
    assert abs(pr - p_ref) < 2e-8 and abs(qr - q_ref) < 1e-4


def test_smallest_extents_match_oracle(m, orc):
    """Extent 2 in every direction (n + mu = n - mu) and mixed 2/4/6 extents:
    FP64 sweeps per link against the oracle."""
    for d in ([2, 2, 2, 2], [2, 4, 2, 6]):
        f = field(m, d)
        m.su3_init_hot(f, 23, 0)
        h = m.su3_sweep_hb_or(f, 6.0, 23, 0, 0, 3, P(n_or=2))
        U = orc.init_hot(d, 23, 0)
        href, _ = orc.sweep_hb_or(d, U, 6.0, 23, 0, 0, 3, n_or=2)
        assert np.max(np.abs(h - href)) < 1e-13, d
        assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 1e-12, d


def test_errors_and_empty_work(m, orc):
    """Validation failures return status codes and leave fields untouched;
    zero sweeps and zero steps are no-ops."""
    import paper_1510_04675_amd as msmc
    for bad in ([3, 4, 4, 4], [4, 4, 0, 4], [1, 2, 2, 2]):
        with pytest.raises(msmc.SU3Error) as e:
            m.Field(bad, "fp64")
        assert e.value.code == 2
    f = field(m, [4, 4, 4, 4])
    m.su3_init_hot(f, 3, 0)
    before = m.su3_field_to_host(f)
    with pytest.raises(msmc.SU3Error) as e:
        m.su3_sweep_hb_or(f, 6.0, 3, 0, 0, 1, P(n_or=-1))
    assert e.value.code == 1
    with pytest.raises(msmc.SU3Error) as e:
        m.su3_sweep_hb_or(f, float("nan"), 3, 0, 0, 1, P())
    assert e.value.code == 1
    coarse = field(m, [2, 2, 2, 4])
    with pytest.raises(msmc.SU3Error) as e:
        m.su3_prolongate(coarse, f)
    assert e.value.code == 2
    with pytest.raises(msmc.SU3Error) as e:
        m.su3_batch_sweep_hb_or([f, f], [6.0, 6.0], [1, 1], [0, 1], 0, 1, P())
    assert e.value.code == 1
    g = field(m, [4, 4, 4, 4], "fp32")
    with pytest.raises(msmc.SU3Error) as e:
        m.su3_batch_sweep_hb_or([f, g], [6.0, 6.0], [1, 1], [0, 1], 0, 1, P())
    assert e.value.code == 6
    with pytest.raises(msmc.SU3Error) as e:
        m.su3_wilson_loop(f, 0, 1)
    assert e.value.code == 1
    with pytest.raises(msmc.SU3Error) as e:
        m.su3_wilson_flow_adaptive(f, 1.0, 0.01, 0.2, 0.01, [0.5, 0.2])
    assert e.value.code == 1
    assert np.array_equal(m.su3_field_to_host(f), before)
    m.su3_sweep_hb_or(f, 6.0, 3, 0, 0, 0, P())
    m.su3_wilson_flow(f, 0.01, 0)
    m.su3_batch_sweep_hb_or([f], [6.0], [3], [0], 0, 0, P())
    assert np.array_equal(m.su3_field_to_host(f), before)


def test_large_lattice_48_4_fp64_sweep_matches_oracle(m, orc):
    """48^4 (5.3 M sites, 3 GB of FP64 links; slabs of 382 MB): one sweep of
    1 HB + 1 OR per link against the oracle, in the benchmark's launch path."""
    d = [48, 48, 48, 48]
    f = field(m, d)
    m.su3_init_hot(f, 29, 0)
    h = m.su3_sweep_hb_or(f, 6.0, 29, 0, 0, 1, P(n_or=1))
    U = orc.init_hot(d, 29, 0)
    href, _ = orc.sweep_hb_or(d, U, 6.0, 29, 0, 0, 1, n_or=1)
    assert abs(h[0] - href[0]) < 1e-13
    assert np.max(np.abs(m.su3_field_to_host(f) - U)) < 1e-12


@pytest.mark.timeout(600)
def test_field_beyond_4_gib_64_4_fp64_sweep_matches_oracle(m, orc):
    """64^4 FP64 (16.8 M sites, a 9.7 GB field whose slabs start beyond 4 GiB,
    so every 32-bit byte offset would wrap): one sweep of 1 HB + 1 OR per
    link against the oracle, compared in slices to bound host memory."""
    d = [64, 64, 64, 64]
    f = field(m, d)
    m.su3_init_hot(f, 31, 0)
    h = m.su3_sweep_hb_or(f, 6.0, 31, 0, 0, 1, P(n_or=1))
    Ug = m.su3_field_to_host(f)
    f.close()
    U = orc.init_hot(d, 31, 0)
    href, _ = orc.sweep_hb_or(d, U, 6.0, 31, 0, 0, 1, n_or=1)
    assert abs(h[0] - href[0]) < 1e-13
    n = Ug.shape[0]
    step = n // 8
    dev = max(float(np.max(np.abs(Ug[i:i + step] - U[i:i + step]))) for i in range(0, n, step))
    assert dev < 1e-12, dev


def test_library_owned_field_and_stream(m, orc):
    """A field the library allocates itself (su3_field_create) on a separate
    HIP stream gives bitwise the result of a torch-wrapped field; info reports
    shape, precision and size; destroy frees it."""
    import ctypes as C

    import torch

    import paper_1510_04675_amd as msmc
    lib = msmc.lib()
    d = [4, 6, 4, 2]
    s = torch.cuda.Stream()
    dims = (C.c_int32 * 4)(*d)
    h = C.c_void_p()
    assert lib.su3_field_create(dims, 2, C.c_void_p(s.cuda_stream), C.byref(h)) == 0

    class Raw:
        handle = h
        volume = int(np.prod(d))

    out_dims = (C.c_int32 * 4)()
    prec, nbytes = C.c_int32(), C.c_size_t()
    assert lib.su3_field_info(h, out_dims, C.byref(prec), C.byref(nbytes)) == 0
    assert list(out_dims) == d and prec.value == 2 and nbytes.value == m.su3_field_bytes(d, 2)
    m.su3_init_hot(Raw, 8, 1)
    hr = m.su3_sweep_hb_or(Raw, 6.0, 8, 1, 0, 2, P(n_or=2, reunit=1))
    f = field(m, d, "fp32_r12")
    m.su3_init_hot(f, 8, 1)
    hf = m.su3_sweep_hb_or(f, 6.0, 8, 1, 0, 2, P(n_or=2, reunit=1))
    assert np.array_equal(hr, hf)
    assert np.array_equal(m.su3_field_to_host(Raw), m.su3_field_to_host(f))
    assert lib.su3_field_destroy(h) == 0
