"""The five workload configurations at their full sizes, through the C ABI.

C1 (4^4, 10 sweeps) is in test_gpu_parity.  Here:
  C2  16^4 cold start, 200 sweeps, FP64 per link against the oracle and the
      FP32 / FP32-R12 chains against the FP64 one;
  C3  8^4 coarse chain -> prolongation -> 16^4 FP32-R12 rethermalization ->
      100 RK3 flow steps -> plaquette and clover charge;
  C4  48 prolongated lattices of three sizes in one batched graph launch;
  C5  HMC on a thermalized 32^4 lattice with FP32 molecular dynamics.
Markov chains in FP32 separate from the FP64 chain by chaos (overrelaxation
amplifies a perturbation about five-fold per pass), so FP32 chains are
compared with the FP64 one on the first sweep, where they still share every
decision, and statistically after thermalization; measurements (plaquette,
flow, charge) are compared on the same field."""
import math
import os
import time

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


def P(n_or=4, hits=1, tries=64, reunit=0, sampler=0):
    import paper_1510_04675_amd as msmc
    return msmc.hb_params(n_or, hits, tries, reunit, sampler)


def sync():
    import torch
    torch.cuda.synchronize()


def binned_mean_err(x, nbins):
    b = np.asarray(x).reshape(nbins, -1).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / math.sqrt(nbins))


@pytest.mark.timeout(600)
def test_config2_16_4_cold_200_sweeps(m, orc):
    """16^4, beta 6.0, cold start, heat-bath seed 2, 200 sweeps of 1 HB +
    4 OR.  FP64: all 200 plaquettes within 1e-13 and every link within 1e-12
    of the oracle.  FP32 (18 reals) and FP32-R12, FP64 reunitarization every
    10 sweeps: the first plaquette within 1e-6 of the FP64 one; after
    thermalization (sweeps 100-199) the mean plaquette equal to the FP64
    chain's within 4 standard errors (10 bins of 10 sweeps per chain)."""
    d = [16] * 4
    f = m.Field(d, "fp64")
    m.su3_init_cold(f)
    t0 = time.perf_counter()
    h64 = m.su3_sweep_hb_or(f, 6.0, 2, 0, 0, 200, P())
    t_gpu = time.perf_counter() - t0
    U = orc.init_cold(d)
    href, ex = orc.sweep_hb_or(d, U, 6.0, 2, 0, 0, 200)
    dl = float(np.max(np.abs(m.su3_field_to_host(f) - U)))
    print(f"\nC2 fp64: {t_gpu:.2f} s for 200 sweeps, max plaquette diff {np.max(np.abs(h64 - href)):.1e}, "
          f"max link diff {dl:.1e}, exhausted {ex}")
    assert np.max(np.abs(h64 - href)) < 1e-13
    assert dl < 1e-12
    ref_mean, ref_err = binned_mean_err(href[100:], 10)
    for prec in ("fp32", "fp32_r12"):
        g = m.Field(d, prec)
        m.su3_init_cold(g)
        h = m.su3_sweep_hb_or(g, 6.0, 2, 0, 0, 200, P(reunit=10))
        dev = np.abs(h - href)
        first = int(np.argmax(dev > 1e-6)) if np.any(dev > 1e-6) else 200
        mean, err = binned_mean_err(h[100:], 10)
        comb = math.hypot(err, ref_err)
        print(f"C2 {prec}: first sweep dP {dev[0]:.1e}, first sweep with dP > 1e-6: {first}, max dP {dev.max():.1e}; "
              f"<P> {mean:.6f}({err:.1e}) vs fp64 {ref_mean:.6f}({ref_err:.1e}), {abs(mean - ref_mean) / comb:.2f} sigma")
        assert dev[0] < 1e-6
        assert abs(mean - ref_mean) < 4 * comb
        ok, mx, _ = m.su3_check_field(g, 1e-5)
        assert ok, mx


@pytest.mark.timeout(900)
def test_config3_multiscale_step(m, orc):
    """8^4 at beta 5.8 (hot start seed 7, 100 sweeps, FP64) -> prolongation
    (c = 0.05, relative tolerance 1e-5) -> 16^4 at beta 6.0, 50 sweeps in
    FP32-R12 (seed 7, first sweep 100) -> 100 RK3 flow steps of eps = 0.01 ->
    plaquette and clover Q.  Coarse chain and prolongation match the oracle
    per link; the R12 chain matches the FP64 one on its first sweep and, after
    25 sweeps, in mean plaquette within 5 single-configuration spreads; the
    R12 flow and its P and Q match the oracle's flow of the same field."""
    dc, df = [8] * 4, [16] * 4
    times = {}
    c = m.Field(dc, "fp64")
    m.su3_init_hot(c, 7, 0)
    t0 = time.perf_counter()
    hc = m.su3_sweep_hb_or(c, 5.8, 7, 0, 0, 100, P())
    times["coarse 100 sweeps"] = time.perf_counter() - t0
    Uc = orc.init_hot(dc, 7, 0)
    hcref, _ = orc.sweep_hb_or(dc, Uc, 5.8, 7, 0, 0, 100)
    assert np.max(np.abs(hc - hcref)) < 1e-13
    assert np.max(np.abs(m.su3_field_to_host(c) - Uc)) < 1e-12

    f64 = m.Field(df, "fp64")
    t0 = time.perf_counter()
    it = m.su3_prolongate(c, f64, 0.05, 1e-5, 10000)
    sync()
    times["prolongation (fp64)"] = time.perf_counter() - t0
    Uf, rit = orc.prolongate(dc, Uc, 0.05, 1e-5, 10000)
    dpro = float(np.max(np.abs(m.su3_field_to_host(f64) - Uf)))
    print(f"\nC3 prolongation: iterations {list(it)} (oracle {list(rit)}), max link diff {dpro:.1e}")
    assert list(it) == list(rit)
    assert dpro < 1e-11
    # partial and displaced averages after prolongation (Sec. III): the displaced
    # 2 x 2 loops from even sites are the coarse plaquettes
    sync()
    t0 = time.perf_counter()
    dl = m.su3_displaced_loops(f64)
    pp = m.su3_partial_plaquettes(f64)
    times["displaced + partial averages (fp64)"] = time.perf_counter() - t0
    print(f"C3 after prolongation: displaced 2x2 {np.round(dl, 6).tolist()}, partial 1x1 {np.round(pp, 6).tolist()}, "
          f"coarse plaquette {hcref[-1]:.6f}")
    assert abs(dl[0] - hcref[-1]) < 1e-13
    for k in range(5):
        assert abs(dl[k] - orc.displaced_2x2(df, Uf, k)) < 1e-13
    for k in range(3):
        assert abs(pp[k] - orc.partial_plaquette(df, Uf, k)) < 1e-13

    fr = m.Field(df, "fp32_r12")
    m.su3_prolongate(c, fr, 0.05, 1e-5, 10000)
    t0 = time.perf_counter()
    hr = m.su3_sweep_hb_or(fr, 6.0, 7, 0, 100, 50, P(reunit=10))
    times["rethermalization 50 sweeps (r12)"] = time.perf_counter() - t0
    dl_after = m.su3_displaced_loops(fr)
    print(f"C3 after rethermalization: displaced 2x2 {np.round(dl_after, 5).tolist()} (spread "
          f"{dl_after.max() - dl_after.min():.1e}, before {dl.max() - dl.min():.1e})")
    assert dl_after.max() - dl_after.min() < 0.2 * (dl.max() - dl.min())
    href, _ = orc.sweep_hb_or(df, Uf, 6.0, 7, 0, 100, 50)
    spread = float(np.std(href[25:]))
    print(f"C3 rethermalization: first sweep dP {abs(hr[0] - href[0]):.1e}; <P>[25:50] r12 {hr[25:].mean():.6f} "
          f"fp64 {href[25:].mean():.6f}, single-config spread {spread:.1e}")
    assert abs(hr[0] - href[0]) < 1e-6
    assert abs(hr[25:].mean() - href[25:].mean()) < 5 * spread

    # flow of this exact field: GPU R12, GPU FP64 and the oracle
    Uh = m.su3_field_to_host(fr)
    g64 = m.Field(df, "fp64")
    m.su3_field_from_host(g64, Uh)
    t0 = time.perf_counter()
    m.su3_wilson_flow(fr, 0.01, 100)
    p_r12, q_r12 = m.su3_plaquette(fr), m.su3_topological_charge(fr)
    times["flow 100 RK3 steps + P, Q (r12)"] = time.perf_counter() - t0
    m.su3_wilson_flow(g64, 0.01, 100)
    p_64, q_64 = m.su3_plaquette(g64), m.su3_topological_charge(g64)
    orc.wilson_flow(df, Uh, 0.01, 100)
    p_ref, q_ref = orc.plaquette(df, Uh), orc.topological_charge(df, Uh)
    d64 = float(np.max(np.abs(m.su3_field_to_host(g64) - Uh)))
    print(f"C3 after flow: P r12 {p_r12:.8f} fp64 {p_64:.10f} oracle {p_ref:.10f}; Q r12 {q_r12:.6f} fp64 {q_64:.8f} "
          f"oracle {q_ref:.8f}; fp64 max link diff {d64:.1e}")
    print("C3 stage times (s): " + ", ".join(f"{k} {v:.3f}" for k, v in times.items()))
    assert d64 < 1e-10
    assert abs(p_64 - p_ref) < 1e-12 and abs(q_64 - q_ref) < 1e-9
    # R12 stores are re-orthonormalized in fp64 and rounded once, so the
    # flowed plaquette carries only rounding noise (about 1e-9 here; an fp32
    # Gram-Schmidt shifted it by 2e-7 through a sign-consistent norm bias)
    assert abs(p_r12 - p_ref) < 2e-8
    assert abs(q_r12 - q_ref) < 1e-4


def c4_lattices(m, prec):
    """48 prolongated lattices: 16 each of 12^4, 16^4, 20^4; beta_i uniform in
    [5.9, 6.2]; coarse (L/2)^4 hot start (seed 4, lattice id i), 20 sweeps at
    beta_i - 0.36, prolongation with c = 0.05 and tolerance 1e-5."""
    sizes = [12] * 16 + [16] * 16 + [20] * 16
    betas = si.batch_betas(48, 4)
    fields = []
    for i, L in enumerate(sizes):
        c = m.Field([L // 2] * 4, "fp64")
        m.su3_init_hot(c, 4, i)
        m.su3_sweep_hb_or(c, betas[i] - 0.36, 4, i, 0, 20, P(), record=False)
        f = m.Field([L] * 4, prec)
        m.su3_prolongate(c, f, 0.05, 1e-5, 10000)
        c.close()
        fields.append(f)
    return sizes, betas, fields


@pytest.mark.timeout(900)
def test_config4_batched_rethermalization(m, orc):
    """48 prolongated lattices of three sizes, FP32 links, 100 sweeps in one
    batched graph launch: per-lattice plaquette histories; three sampled
    lattices rerun alone give bitwise the same fields and histories; the first
    sweep of a 12^4 member matches the FP64 oracle from the same field within
    1e-6; thermalized plaquettes increase with beta (rank correlation > 0.95)."""
    sizes, betas, fs = c4_lattices(m, "fp32")
    start12 = m.su3_field_to_host(fs[3])
    seeds = [4] * 48
    lids = list(range(48))
    sync()
    t0 = time.perf_counter()
    h = m.su3_batch_sweep_hb_or(fs, betas, seeds, lids, 0, 100, P(reunit=10))
    dt = time.perf_counter() - t0
    links = sum(4 * L ** 4 for L in sizes)
    print(f"\nC4: {len(fs)} lattices, {links} links, 100 sweeps in {dt:.3f} s = {5 * links * 100 / dt:.3e} link updates/s")
    # sampled lattices alone, from the same prolongated starts
    _, _, gs = c4_lattices(m, "fp32")
    for i in (0, 17, 40):
        hs = m.su3_sweep_hb_or(gs[i], betas[i], 4, i, 0, 100, P(reunit=10))
        assert np.array_equal(hs, h[:, i]), i
        assert np.array_equal(m.su3_field_to_host(gs[i]), m.su3_field_to_host(fs[i])), i
    # first sweep of lattice 3 (12^4) against the oracle
    U = start12.copy()
    href, _ = orc.sweep_hb_or([12] * 4, U, betas[3], 4, 3, 0, 1)
    print(f"C4 lattice 3 first sweep: gpu {h[0, 3]:.8f} oracle {href[0]:.8f}")
    assert abs(h[0, 3] - href[0]) < 1e-6
    # physics: thermalized plaquette rises with beta
    pm = h[50:].mean(axis=0)
    rb = np.argsort(np.argsort(betas))
    rp = np.argsort(np.argsort(pm))
    rho = 1 - 6 * np.sum((rb - rp) ** 2) / (48 * (48 ** 2 - 1))
    print(f"C4 plaquettes: {np.round(pm, 5).tolist()}; rank correlation with beta {rho:.3f}")
    assert rho > 0.95
    for f in fs + gs:
        f.close()


@pytest.mark.timeout(900)
def test_config5_hmc_32_4(m, orc):
    """32^4, beta 6.0, thermalized start (cold + 200 HB+OR sweeps, seed 5).
    A short FP64 trajectory (4 steps of eps = 0.025) matches the oracle in dH
    (to 1e-6: H ~ 3e7 is summed in different orders), decision and links; one full trajectory (tau 1, 40 steps) in FP32 gives
    dH close to the FP64 one from the same start; 20 FP32 trajectories give an
    acceptance consistent with erfc(sqrt(<dH>)/2) and a plaquette consistent
    with the heat-bath value."""
    d = [32] * 4
    f = m.Field(d, "fp64")
    m.su3_init_cold(f)
    hh = m.su3_sweep_hb_or(f, 6.0, 5, 0, 0, 200, P())
    p_hb = float(hh[150:].mean())
    spread = float(np.std(hh[150:]))
    U = m.su3_field_to_host(f)
    acc, dH = m.su3_hmc_trajectory(f, 6.0, 0.1, 4, 5, 0, 1000, 1)
    racc, rdH = orc.hmc_trajectory(d, U, 6.0, 0.1, 4, 5, 0, 1000, 1)
    dl = float(np.max(np.abs(m.su3_field_to_host(f) - U)))
    print(f"\nC5 fp64 short trajectory: dH {dH:.10f} oracle {rdH:.10f}, accepted {acc}/{racc}, max link diff {dl:.1e}")
    # H is a sum of ~3e7 terms of order 1 (|H| ~ 3e7); the GPU adds them in
    # a fixed tree (error about log2(n) ulps of the total, ~1e-7) and the
    # oracle with compensated summation, so dH agrees to about 1e-7.
    assert acc == racc
    assert abs(dH - rdH) < 1e-6
    assert dl < 1e-11

    # FP64 vs FP32 molecular dynamics on one full trajectory from the same start
    m.su3_field_from_host(f, U)
    g = m.Field(d, "fp32")
    m.su3_field_from_host(g, U)
    _, dh64 = m.su3_hmc_trajectory(f, 6.0, 1.0, 40, 5, 0, 0, 0)
    _, dh32 = m.su3_hmc_trajectory(g, 6.0, 1.0, 40, 5, 0, 0, 0)
    print(f"C5 one trajectory from the same start: dH fp64 {dh64:.6f} fp32 {dh32:.6f}")
    assert abs(dh32 - dh64) < 0.05 + 0.02 * abs(dh64)

    # 20 FP32 trajectories with Metropolis
    m.su3_field_from_host(g, U)
    sync()
    t0 = time.perf_counter()
    dhs, n_acc = [], 0
    for t in range(20):
        a, x = m.su3_hmc_trajectory(g, 6.0, 1.0, 40, 5, 0, 1 + t, 1)
        n_acc += a
        dhs.append(x)
    dt = time.perf_counter() - t0
    mdh = float(np.mean(dhs))
    pred = math.erfc(0.5 * math.sqrt(max(mdh, 0.0)))
    p_hmc = m.su3_plaquette(g)
    print(f"C5 20 trajectories: {20 / dt:.2f} traj/s, acceptance {n_acc / 20:.2f} (erfc model {pred:.3f}), "
          f"<dH> {mdh:.4f}, <exp(-dH)> {np.mean(np.exp(-np.array(dhs))):.4f}, plaquette {p_hmc:.6f} "
          f"(heat bath {p_hb:.6f})")
    sd = math.sqrt(pred * (1 - pred) / 20)
    assert abs(n_acc / 20 - pred) < 3 * sd + 0.05
    assert abs(p_hmc - p_hb) < 5 * spread
