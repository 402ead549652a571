"""Benchmark: batched log-likelihood + gradient evaluations per second on one MI355X.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-cpu-baseline]

Workload (synthetic, seed-fixed): EPL + shear lens, Sersic lens light, Sersic + shapelet
(n_max = 6) source on a 60 x 60 image at 0.065"/px, 2x supersampled, Moffat 21 x 21 PSF,
4096 parameter vectors (2048 near the seed truth, 2048 from a broadened prior); the
observed image is the stored seed-0 image written by the oracle. A step is one
gl_loglik_grad call over the 4096 vectors (decode, sub-pixel forward, PSF + likelihood,
adjoint), with inputs resident in HBM.

Prints one JSON line: the metric, the roofline of the dominant kernel (algorithmic FLOPs of
the op-count model below over its HIP-event duration), the FP64 oracle timed on the host
cores on a bounded sample, a serving stream against the serial loop, and the wall time of
the whole modelling pipeline of one system (multi-start Adam -> VI -> HMC).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (256 CU x 2.4 GHz x 256 FLOP/clk)
SERIES_TOL_FP32 = 6e-8     # series length counted by the op model (FP32 resolution)
# the kernels behind each stage (rocprofv3 kernel names)
KERNEL_NAMES = {"subpix_adj": "subpix_adj_kernel", "subpix_fwd": "subpix_fwd_kernel",
                "conv_lik": "conv_mfma_kernel"}

# ------------------------------------------------------------------------------------------
# Algorithmic op-count model (frozen; FMA = 2, add / mul / compare = 1, each transcendental
# (exp, log, sqrt, reciprocal, atan) = 1). Counts follow the formulas of the model as written
# out in the forward and adjoint equations, per unit of work:
#   sub-pixel forward:  mass 52 + 7 N(eps) [N = series terms at FP32 resolution],
#                       Sersic 16 (+2 lens offsets), shapelets 2 + 2(1 + 4(n-1)) + 3M + 6,
#                       sum + downsample 3
#   pixel:              PSF 2 K^2, likelihood 11, adjoint seed 7, adjoint PSF 2 K^2, scale 1
#   sub-pixel adjoint:  mass 52 + 21 N + 142, source Sersic 52, lens Sersic 58,
#                       shapelets 49 + 11 M + 16 (n = n_max, M coefficients), centre 6, 2
# ------------------------------------------------------------------------------------------

def series_terms(eps_abs: np.ndarray) -> np.ndarray:
    e = np.clip(np.asarray(eps_abs, np.float64), 1e-30, 0.6)
    n = np.ceil(np.log(SERIES_TOL_FP32 * (1 - e)) / np.log(e))
    return np.clip(n, 1, None)


def flops_model(H, W, k, K, nmax, lens_light, N_mean, sie=False):
    M = 0 if nmax < 0 else (nmax + 1) * (nmax + 2) // 2
    S, Px = H * W * k * k, H * W
    mass_f = 52 + 7 * N_mean
    shp_f = 0 if nmax < 0 else 2 + 2 * (1 + 4 * max(nmax - 1, 0)) + 3 * M + 6
    sub_f = mass_f + 16 + (18 if lens_light else 0) + shp_f + 3
    mass_a = 52 + 21 * N_mean + 142
    shp_a = 0 if nmax < 0 else 49 + 11 * M + 16
    sub_a = mass_a + 52 + (58 if lens_light else 0) + shp_a + 6 + 2
    return {
        "subpix_fwd": S * sub_f,
        "conv_lik": Px * (2 * K * K + 11),
        "conv_lik_adj": Px * (2 * K * K + 11 + 7 + 2 * K * K + 1),
        "subpix_adj": S * sub_a,
    }


# ------------------------------------------------------------------------------------------

# the translation unit the likelihood and adjoint kernels are compiled in, with every file it
# includes: a change to any of them can change the profiled kernels' code
KERNEL_SOURCES = ["paper_2202_07663_amd/csrc/" + f for f in (
    "glens_api.hip", "glens_kernels.h", "glens_particle.h", "glens_device.h",
    "glens_fit_device.h", "glens_types.h", "glens_host.h")] + ["include/gl.h"]


def csrc_hash() -> str:
    """Hash of the likelihood kernels' sources (a profile record is used only while it holds)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def load_profile(workload: str):
    """The committed rocprofv3 record of this workload (kernel-trace durations, HBM counters
    scaled by the copy calibration, VALU instruction counters per sub-pixel), or None when
    the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"record_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("csrc_hash") != csrc_hash():
        return None
    return rec


def executed_flop_per_subpixel(counters: dict) -> float:
    """FLOP a kernel executes per sub-pixel from its VALU instruction counters (wave
    instructions x 64 lanes per sub-pixel): FMA = 2, add / mul / transcendental = 1, in FP32
    and FP64. Moves, conversions, compares and selects are not arithmetic and not counted."""
    c = counters
    return (2 * c["SQ_INSTS_VALU_FMA_F32"] + c["SQ_INSTS_VALU_ADD_F32"] + c["SQ_INSTS_VALU_MUL_F32"]
            + c["SQ_INSTS_VALU_TRANS_F32"] + 2 * c["SQ_INSTS_VALU_FMA_F64"]
            + c["SQ_INSTS_VALU_ADD_F64"] + c["SQ_INSTS_VALU_MUL_F64"] + c["SQ_INSTS_VALU_TRANS_F64"])


def cpu_info() -> dict:
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


def call_times_ms(fn, n):
    """Durations of n back-to-back calls (ms), from HIP events on the current stream (the
    library's kernels run on it)."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in ev])


def spread(ms: np.ndarray, P: int) -> dict:
    q = np.percentile(ms, [10, 50, 90])
    return {"calls": int(ms.size), "ms_p10": round(float(q[0]), 4), "ms_median": round(float(q[1]), 4),
            "ms_p90": round(float(q[2]), 4), "evals_per_s_median": round(P / (q[1] * 1e-3), 1)}


def stored(spec, seed=0):
    """The stored observed image (written by the oracle) and seed truth of a workload."""
    obs = np.load(os.path.join(ROOT, "tests", "golden", f"obs_{spec.name}_s{seed}.npy"))
    truth = np.load(os.path.join(ROOT, "tests", "golden", f"truth_{spec.name}_s{seed}.npy"))
    return obs, truth


def workload():
    import synth
    spec = synth.spec_c2()
    obs, truth = stored(spec)
    theta = synth.draw_particles(spec, truth, 4096, seed=0)
    return spec, obs, theta


# ------------------------------------------------------------------------------------------
# The modelling pipeline of one system (Table 1): multi-start Adam (n_MAP starts x K_MAP
# steps, lr 1e-2 -> 1e-3 linear), VI (n_VI samples x K_VI iterations, lr 0 -> 1e-3
# quadratic over 500, Sigma_1 = 1e-6 I, from the best start), then HMC (chains drawn from the
# VI surrogate, 250 burn-in + 750 recorded trajectories starting at L leapfrog steps of
# eps_0 = 0.3, with the step size (acceptance 0.75) and the trajectory length (ChEES, at most
# 100 steps) adapted over 80% of burn-in, M^-1 = the VI covariance). Every stage
# runs on the GPU; each is timed from its first launch to a device sync. One system, the
# paper's simulated-system setting (eq. sim-dist truth and prior, 80x80, k = 2, sigma_bkg 0.2,
# t_exp 100 s; truth seed 6, whose arcs have the typical signal-to-noise of about 100 the
# paper quotes), in two configurations:
#   pipeline:      Table 1's sizes (300 x 300, 500 x 1000, 50 chains x L = 5);
#   pipeline_long: 6000 surrogate iterations at rate 3e-3 from sd 3e-3, and 1000 burn-in +
#                  1000 recorded trajectories.
# ------------------------------------------------------------------------------------------

def pipeline_bench(spec, obs, truth, seed=0, n_map=4096, k_map=300, n_vi=1000, k_vi=1000,
                   chains=64, L=10, n_burn=250, n_samples=750, max_leapfrog=100,
                   adapt_length=True, vi_lr=1e-3, vi_warmup=500, vi_init_sd=1e-3,
                   map_result=None, vi_lr_final=0.0, adapt_mass=False, full=False,
                   priors=None):
    """map_result: (fit result, seconds) of a MAP stage already run with these settings (the
    stage is then not run again; its time is reported as measured there). full: also return
    the posterior means and standard deviations, split R-hat and ESS of every parameter."""
    import torch
    import synth
    import paper_2202_07663_amd as G
    from paper_2202_07663_amd import diagnostics as dg
    if priors is None:
        priors = synth.fit_priors(spec)
    model = G.Model.from_spec(spec, obs)
    torch.cuda.synchronize()
    if map_result is None:
        t0 = time.perf_counter()
        r = G.fit(model, n_map, k_map, priors, seed=seed)
        t1 = time.perf_counter()
    else:
        r, dt_map = map_result
        t1 = time.perf_counter()
        t0 = t1 - dt_map
    vi = G.VI(model, n_vi, k_vi, priors, r["z_best"].astype(np.float64), lr_max=vi_lr,
              lr_warmup=vi_warmup, init_sd=vi_init_sd, seed=seed + 1, lr_final=vi_lr_final)
    vi.step()
    got = vi.get()
    z0 = vi.sample(chains, seed=seed + 2)
    chol = got["chol"].cpu().numpy()
    t2 = time.perf_counter()
    h = G.HMC(model, chains, L, n_burn, n_samples, priors, step_size=0.3, seed=seed + 3,
              z0=z0, mass_chol=chol, adapt_length=adapt_length, max_leapfrog=max_leapfrog,
              adapt_mass=adapt_mass)
    h.run()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    info = h.info()
    th = h.samples().cpu().numpy().astype(np.float64)  # [n_samples, chains, d]
    flat = th.reshape(-1, th.shape[-1])
    mean, sd = flat.mean(axis=0), flat.std(axis=0)
    pull = np.abs(mean - truth) / np.maximum(sd, 1e-30)
    rhat, ess = dg.split_rhat(th), dg.ess(th)
    names = model.names
    light = {n: [round(float(mean[j]), 5), round(float(sd[j]), 5), round(float(truth[j]), 5)]
             for j, n in enumerate(names) if not (n.startswith("c") and n[1:].isdigit())}
    grad_evals = n_map * k_map + n_vi * k_vi + round(chains * (n_burn + n_samples) *
                                                     info["mean_leapfrog"])
    return {
        "config": {"map": [n_map, k_map],
                   "vi": [n_vi, k_vi, vi_lr, vi_init_sd] + ([vi_lr_final] if vi_lr_final else []),
                   "hmc": {"chains": chains, "L": L, "burn": n_burn, "samples": n_samples,
                           **({"adapt_mass": True} if adapt_mass else {})}},
        "seconds": {"map": round(t1 - t0, 3), "vi": round(t2 - t1, 3), "hmc": round(t3 - t2, 3),
                    "total": round(t3 - t0, 3)},
        "grad_evals": grad_evals,
        "grad_evals_per_s": round(grad_evals / (t3 - t0), 1),
        "hmc_us_per_leapfrog": round(1e6 * (t3 - t2) / ((n_burn + n_samples) *
                                                        info["mean_leapfrog"]), 2),
        "hmc_trajectory_length": round(info["trajectory_length"], 4),
        "hmc_mean_leapfrog": round(info["mean_leapfrog"], 2),
        "hmc_mass_updates": info["mass_updates"],
        "map_chi2nu": round(r["chi2nu"], 4),
        "hmc_accept": round(info["accept_mean"], 4),
        "hmc_step_size": info["step_size"],
        "rhat_max": round(float(np.max(rhat)), 4),
        "ess_min": round(float(np.min(ess)), 1),
        "ess_per_s_hmc": round(float(np.min(ess)) / (t3 - t2), 1),
        "truth_pull_median": round(float(np.median(pull)), 3),
        "truth_pull_max": round(float(np.max(pull)), 3),
        "posterior_mean_sd_truth": light,
        **({"post_mean": mean.tolist(), "post_sd": sd.tolist(), "rhat": np.asarray(rhat).tolist(),
            "ess": np.asarray(ess).tolist(), "post_median": np.median(flat, axis=0).tolist(),
            "map_theta": np.asarray(r["theta_best"], np.float64).tolist(),
            "truth_rank": np.mean(flat < truth[None, :], axis=0).tolist()} if full else {}),
        "paper_context": "Table 1: 17 s + 52 s + 36 s = 105 s on 4x A100 (about 6 min on one) "
                         "for the paper's reference system (another PSF and truth)",
    }


def vi_estimator_bench(seed=1000):
    """Table 1's VI budget (500 draws x 1000 iterations, rate 0 -> 1e-3 over 500) from the MAP
    point of one system drawn from the paper's simulation distribution, once with each
    gradient estimator: seconds, the loss at the start, around iteration 500 and over the
    last 50 iterations, and the surrogate's standard deviations."""
    import torch
    import synth
    import paper_2202_07663_amd as G
    sp = synth.spec_paper80()
    truth = synth.draw_truth(sp, seed)
    sim = G.Model.from_spec(sp)
    clean = sim.simulate(torch.from_numpy(truth[None, :]).cuda())[0].cpu().numpy()
    sim.close()
    obs = synth.add_noise(clean, seed, sp.sigma_bkg, sp.t_exp)
    pri = synth.fit_priors(sp)
    model = G.Model.from_spec(sp, obs)
    r = G.fit(model, 2048, 2000, pri, seed=seed)
    out = {"workload": f"paper80 (eq. sim-dist draw, seed {seed}), MAP 2048 x 2000",
           "map_chi2nu": round(r["chi2nu"], 4)}
    for est in ("pathwise", "score"):
        vi = G.VI(model, 500, 1000, pri, r["z_best"].astype(np.float64), lr_max=1e-3,
                  lr_warmup=500, init_sd=1e-3, seed=seed + 1, estimator=est)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vi.step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        loss = vi.get_state()["loss"].cpu().numpy()
        sd = np.sqrt(np.diag(vi.get()["cov"].cpu().numpy()))
        out[est] = {"seconds": round(dt, 3), "loss_first": round(float(loss[0]), 2),
                    "loss_490_510": round(float(np.nanmean(loss[490:510])), 2),
                    "loss_last50": round(float(np.nanmean(loss[-50:])), 2),
                    "sd_min": float(sd.min()), "sd_median": float(np.median(sd)),
                    "sd_max": float(sd.max())}
    return out


def recovery_bench(n_systems, seed0=1000, adapt_mass=True, n_map=300, k_map=300,
                   prior="paper", noise="poisson"):
    """The pipeline at Table 1's sizes on n_systems systems drawn from the paper's simulation
    distribution (eq. sim-dist; the 80x80 configuration of its Sec. 3), each observed as a
    GPU-simulated image plus seeded noise: per parameter the mean and spread of the scaled
    errors z = (posterior mean - truth) / posterior sd, the share of truths within one and
    two posterior sd, the largest split R-hat and the smallest ESS over the systems (the
    statistics of the paper's Table 2). n_map, k_map: the MAP stage's starts and steps.
    prior: "paper" (the broadened prior of eq. sim-dist, as the paper fits) or "sim" (the
    simulation distribution itself, under which the posterior is calibrated by construction).
    noise: "poisson" (shot noise plus Gaussian background, Sec. 2.1.2) or "gauss" (Gaussian
    of the likelihood's own variance). Besides the posterior mean, the scaled errors of the
    posterior median and of the MAP point and the truth's rank among the samples are kept,
    which separate a shift of the whole posterior from its skewness."""
    import torch
    import synth
    import paper_2202_07663_amd as G
    sp = synth.spec_paper80()
    zs, rh, es, secs, chi, acc, zmed, zmap, ranks = [], [], [], [], [], [], [], [], []
    names = None
    for i in range(n_systems):
        seed = seed0 + i
        truth = synth.draw_truth(sp, seed)
        sim = G.Model.from_spec(sp)
        names = sim.names
        clean = sim.simulate(torch.from_numpy(truth[None, :]).cuda())[0].cpu().numpy()
        sim.close()
        if noise == "poisson":
            obs = synth.add_noise(clean, seed, sp.sigma_bkg, sp.t_exp)
        else:
            obs = synth.add_gaussian_noise(clean, seed, sp.sigma_bkg, sp.t_exp)
        r = pipeline_bench(sp, obs, truth, seed=seed, n_map=n_map, k_map=k_map, n_vi=500,
                           k_vi=1000, chains=50, L=5, adapt_mass=adapt_mass, full=True,
                           priors=synth.fit_priors(sp, matched=(prior == "sim")))
        sd = np.maximum(np.asarray(r["post_sd"]), 1e-30)
        zs.append((np.asarray(r["post_mean"]) - truth) / sd)
        zmed.append((np.asarray(r["post_median"]) - truth) / sd)
        zmap.append((np.asarray(r["map_theta"]) - truth) / sd)
        ranks.append(r["truth_rank"])
        rh.append(r["rhat"])
        es.append(r["ess"])
        secs.append(r["seconds"]["total"])
        chi.append(r["map_chi2nu"])
        acc.append(r["hmc_accept"])
        print(f"recovery {i + 1}/{n_systems}: chi2nu {r['map_chi2nu']:.3f} "
              f"rhat {max(r['rhat']):.3f} |z| max {np.abs(zs[-1]).max():.2f}", file=sys.stderr,
              flush=True)
    z, rh, es = np.asarray(zs), np.asarray(rh), np.asarray(es)
    zmed, zmap, ranks = np.asarray(zmed), np.asarray(zmap), np.asarray(ranks)
    per = {n: {"mu_z": round(float(z[:, j].mean()), 3), "sd_z": round(float(z[:, j].std()), 3),
               "mu_z_median": round(float(zmed[:, j].mean()), 3),
               "mu_z_map": round(float(zmap[:, j].mean()), 3),
               "mean_rank": round(float(ranks[:, j].mean()), 3),
               "within_1sd": round(float(np.mean(np.abs(z[:, j]) < 1)), 3),
               "max_rhat": round(float(rh[:, j].max()), 4),
               "min_ess": round(float(es[:, j].min()), 1)} for j, n in enumerate(names)}
    return {
        "workload": "paper80 (eq. sim-dist draws, seeds %d-%d)" % (seed0, seed0 + n_systems - 1),
        "systems": n_systems,
        "prior": prior, "noise": noise,
        "config": {"map": [n_map, k_map], "vi": [500, 1000], "hmc": {"chains": 50, "L0": 5,
                   "burn": 250, "samples": 750, "adapt_length": True,
                   "adapt_mass": bool(adapt_mass)}},
        "seconds_per_system": {"mean": round(float(np.mean(secs)), 3),
                               "max": round(float(np.max(secs)), 3)},
        "map_chi2nu": {"median": round(float(np.median(chi)), 4),
                       "max": round(float(np.max(chi)), 4)},
        "hmc_accept_mean": round(float(np.mean(acc)), 4),
        "within_1sd": round(float(np.mean(np.abs(z) < 1)), 4),
        "within_2sd": round(float(np.mean(np.abs(z) < 2)), 4),
        "abs_mu_z_max": round(float(np.abs(z.mean(axis=0)).max()), 3),
        "max_rhat": round(float(rh.max()), 4),
        "systems_rhat_below_1_05": int(np.sum(rh.max(axis=1) < 1.05)),
        "min_ess": round(float(es.min()), 1),
        "per_parameter": per,
        "paper_context": "Sec. 3, Table 2: 100 systems, largest R-hat 1.017, smallest ESS 26 822",
    }


def cpu_baseline(spec, obs, theta, n_sample: int, n_one: int = 8):
    """The FP64 oracle (dual-number gradient for log L + gradient, plain FP64 for log L alone)
    on evenly spaced vectors of the same batch: all host cores on n_sample vectors, one core
    on n_one."""
    import oracle
    from tests.helpers import oracle_model
    om = oracle_model(spec)
    idx = np.linspace(0, theta.shape[0] - 1, n_sample).astype(int)
    th = theta[idx].astype(np.float64)
    cores = oracle.num_threads()

    def timed(fn, x):
        t0 = time.perf_counter()
        fn(om, x, obs)
        return time.perf_counter() - t0

    t_grad = timed(oracle.loglik_grad, th)
    t_ll = timed(oracle.loglik, th)
    oracle.set_num_threads(1)
    try:
        t_grad1 = timed(oracle.loglik_grad, th[:n_one])
        t_ll1 = timed(oracle.loglik, th[:4 * n_one])
    finally:
        oracle.set_num_threads(cores)
    return {"value": n_sample / t_grad, "unit": "logL+grad evals/s", "cores": cores,
            "kind": "oracle", "seconds": round(t_grad, 3),
            "sample": f"{n_sample} of the 4096 vectors (evenly spaced), same image and model",
            "loglik_only_evals_per_s": round(n_sample / t_ll, 2),
            "one_core": {"logL+grad_evals_per_s": round(n_one / t_grad1, 3),
                         "loglik_only_evals_per_s": round(4 * n_one / t_ll1, 2),
                         "sample": f"the first {n_one} (log L + gradient) and {4 * n_one} "
                                   "(log L) of those vectors"},
            **cpu_info()}


# ------------------------------------------------------------------------------------------
# Serving: a stream of systems of mixed image size and component set (sizes {40, 60, 80,
# 100} px at k = 2 with a Moffat 21 x 21 PSF; SIE or EPL; lens light on or off; shapelets
# none / n_max 4, 6, 8; P a multiple of 256 in [512, 4096]; fixed Adam budget K). The
# observed images come from gl_simulate of a seeded truth plus seeded noise.
# ------------------------------------------------------------------------------------------

def make_stream(n, seed, G, small=False, tiny=False):
    """n requests of the mixed stream (sizes {40, 60, 80, 100} px, k = 2, P a multiple of 256
    in [512, 4096]); with small=True of the smaller systems of that range (sizes {40, 48, 56,
    60} px, P in {512, 768, 1024}); with tiny=True of systems whose launches alone leave most
    of the GPU idle (sizes {32, 40} px, k = 1, P in {64, 128, 256}). Component sets mixed."""
    import synth
    import torch
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        N = int(rng.choice([32, 40] if tiny else ([40, 48, 56, 60] if small else [40, 60, 80, 100])))
        epl = bool(rng.integers(2))
        ll = bool(rng.integers(2))
        nmax = int(rng.choice([-1, 4, 6, 8]))
        P = int(rng.choice([64, 128, 256])) if tiny else \
            int(256 * (rng.integers(2, 5) if small else rng.integers(2, 17)))
        spec = synth.spec_custom(N, 1 if tiny else 2, epl, ll, nmax, K=21)
        truth = synth.draw_truth(spec, 1000 + i)
        m = G.Model.from_spec(spec, None)
        clean = m.simulate(torch.from_numpy(truth[None, :]).cuda()).cpu().numpy()[0]
        m.close()
        obs = synth.add_noise(clean, 1000 + i, spec.sigma_bkg, spec.t_exp)
        out.append((spec, obs, P, synth.fit_priors(spec)))
    return out


def _replay(stream, arrivals, start, done):
    """Submit stream[i] at arrivals[i] seconds (a thread of its own): start(i) queues it;
    done() collects (i, t_submit_s, t_done_s) for every request once all are queued."""
    import threading
    t0 = time.perf_counter()

    def submitter():
        for i in range(len(stream)):
            wait = arrivals[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            start(i)
            _progress("submitted", i + 1, len(stream))

    th = threading.Thread(target=submitter)
    th.start()
    res = done(th)
    return time.perf_counter() - t0, res


def _progress(what, i, n):
    """A line on stderr every 50 systems of a long stream (the JSON line stays alone on
    stdout)."""
    if n >= 100 and (i % 50 == 0 or i == n):
        print(f"{what} {i}/{n} at {time.strftime('%H:%M:%S')}", file=sys.stderr, flush=True)


def serve_stream(G, stream, K, arrivals, steps_per_tick, max_systems):
    """The continuous-batching server: returns (makespan s, latencies s, results, stats)."""
    srv = G.Server(hbm_budget_bytes=96 << 30, max_systems=max_systems,
                   steps_per_tick=steps_per_tick)
    tickets = [None] * len(stream)

    def start(i):
        spec, obs, P, pri = stream[i]
        tickets[i] = srv.submit(spec, obs, P, K, pri, seed=7)

    def done(th):
        th.join()
        out = []
        for i, t in enumerate(tickets):
            out.append(srv.wait(t))
            _progress("served", i + 1, len(tickets))
        return out

    makespan, res = _replay(stream, arrivals, start, done)
    st = srv.stats()
    srv.close()
    assert all(r["status"] == 0 for r in res), [r["status"] for r in res]
    lat = np.array([(r["t_done"] - r["t_submit"]) * 1e-9 for r in res])
    return makespan, lat, res, st


def serial_stream(G, stream, K, arrivals):
    """The plain loop under the same arrivals: one worker takes requests first come first
    served and runs each fit to completion (model creation, gl_fit, teardown)."""
    import queue
    q = queue.Queue()
    t_sub, t_done, res = {}, {}, {}

    def start(i):
        t_sub[i] = time.perf_counter()
        q.put(i)

    def done(th):
        for _ in range(len(stream)):
            i = q.get()
            spec, obs, P, pri = stream[i]
            m = G.Model.from_spec(spec, obs)
            res[i] = G.fit(m, P, K, pri, seed=7)
            m.close()
            t_done[i] = time.perf_counter()
            _progress("serial", len(t_done), len(stream))
        th.join()
        return None

    makespan, _ = _replay(stream, arrivals, start, done)
    assert all(res[i]["status"] == 0 for i in range(len(stream)))
    lat = np.array([t_done[i] - t_sub[i] for i in range(len(stream))])
    return makespan, lat, [res[i] for i in range(len(stream))]


def serving_poisson_bench(n_systems, K, seed=0, steps_per_tick=10, max_systems=16,
                          pilot=50, rate=None, side="both"):
    """A long stream at stable load: the plain loop's service rate from its first `pilot`
    systems (or the given arrival rate), then the server and / or the plain loop under the
    same Poisson arrivals at 0.8 x that rate (no burst runs). side: "both", "served" or
    "serial" (a stream too long for one run is measured one side per run, under the same
    arrival times)."""
    import paper_2202_07663_amd as G
    stream = make_stream(n_systems, seed, G)
    if rate is None:
        pil_span, _, _ = serial_stream(G, stream[:pilot], K, np.zeros(pilot))
        lam = 0.8 * pilot / pil_span
    else:
        lam, pilot = float(rate), 0
    arr = np.cumsum(np.random.default_rng(seed + 1).exponential(1.0 / lam, len(stream)))
    q = lambda x, p: round(float(np.percentile(x, p)), 4)  # noqa: E731
    out = {"stream": "mixed (40-100 px, P 512-4096), Poisson arrivals", "systems": len(stream),
           "K": K, "poisson_rate_per_s": round(lam, 4), "pilot_systems": pilot, "side": side}
    if side in ("both", "served"):
        span, lat, _, st = serve_stream(G, stream, K, arr, steps_per_tick, max_systems)
        out.update({"makespan_s_served": round(span, 2),
                    "fits_per_hour_served": round(3600 * len(stream) / span, 1),
                    "p50_latency_s": q(lat, 50), "p99_latency_s": q(lat, 99),
                    "hbm_peak_bytes": int(st["hbm_peak"])})
    if side in ("both", "serial"):
        ser_span, ser_lat, _ = serial_stream(G, stream, K, arr)
        out.update({"makespan_s_serial": round(ser_span, 2),
                    "fits_per_hour_serial": round(3600 * len(stream) / ser_span, 1),
                    "p50_latency_serial_s": q(ser_lat, 50),
                    "p99_latency_serial_s": q(ser_lat, 99)})
    return out


def serving_bench(n_systems, K, seed=0, steps_per_tick=10, max_systems=16, small=False,
                  tiny=False):
    """Served against the plain loop on the same requests: a burst (all at t = 0: throughput)
    and Poisson arrivals at 0.8 x the plain loop's service rate (latency at stable load), each
    run for real by both; the plain loop's rate is taken from its own burst run."""
    import paper_2202_07663_amd as G
    stream = make_stream(n_systems, seed, G, small, tiny)
    burst = np.zeros(len(stream))
    ser_span, ser_lat_b, ser_res = serial_stream(G, stream, K, burst)
    span, lat_b, res_b, st_b = serve_stream(G, stream, K, burst, steps_per_tick, max_systems)
    mu_serial = len(stream) / ser_span
    lam = 0.8 * mu_serial
    arr = np.cumsum(np.random.default_rng(seed + 1).exponential(1.0 / lam, len(stream)))
    _, lat, _, _ = serve_stream(G, stream, K, arr, steps_per_tick, max_systems)
    _, ser_lat, _ = serial_stream(G, stream, K, arr)
    same = all(a["best"] == b["best"] and a["logpost_best"] == b["logpost_best"]
               for a, b in zip(res_b, ser_res))
    q = lambda x, p: round(float(np.percentile(x, p)), 4)  # noqa: E731
    sub = sum(sp.H * sp.W * sp.k ** 2 * P for sp, _, P, _ in stream) / len(stream)
    return {
        "stream": ("tiny (32-40 px, k 1, P 64-256)" if tiny else
                   "small (40-60 px, P 512-1024)" if small else "mixed (40-100 px, P 512-4096)"),
        "systems": len(stream), "K": K, "steps_per_tick": steps_per_tick,
        "max_systems": max_systems, "mean_subpixels_per_step": round(sub),
        "fits_per_hour_served": round(3600 * len(stream) / span, 1),
        "fits_per_hour_serial": round(3600 * mu_serial, 1),
        "throughput_gain": round(ser_span / span, 3),
        "poisson_rate_per_s": round(lam, 4),
        "p50_latency_s": q(lat, 50), "p99_latency_s": q(lat, 99),
        "p50_latency_serial_s": q(ser_lat, 50), "p99_latency_serial_s": q(ser_lat, 99),
        "burst_p50_s": q(lat_b, 50), "burst_p99_s": q(lat_b, 99),
        "burst_p50_serial_s": q(ser_lat_b, 50), "burst_p99_serial_s": q(ser_lat_b, 99),
        "results_equal_served_and_serial": bool(same),
        "hbm_peak_bytes": int(st_b["hbm_peak"]),
    }


def c4_bench(G, spec):
    """The whole fit of the 60x60 EPL + shapelet system (stored observation, seed 0): 4096
    starts, VI 1000 x 1000, HMC 64 chains x (250 + 750) trajectories x 10 leapfrog steps, as
    the paper runs it and with the mass matrix re-estimated during burn-in; then the same MAP
    point with a longer surrogate fit whose rate decays, and longer chains; last, the whole
    fit from 512 starts with the mass-adapted chains."""
    import torch
    import synth
    # At this signal-to-noise (sigma_bkg 0.1, t_exp 1000 s) and d = 51 the multi-start Adam
    # needs ~1e4 steps to reach the global mode; Table 1's 300 steps are run and reported
    # beside it.
    obs0, truth0 = stored(spec, 0)
    m0 = G.Model.from_spec(spec, obs0)
    t0 = time.perf_counter()
    r300 = G.fit(m0, 4096, 300, synth.fit_priors(spec), seed=0)
    torch.cuda.synchronize()
    map300 = {"K": 300, "P": 4096, "chi2nu": round(r300["chi2nu"], 4),
              "seconds": round(time.perf_counter() - t0, 3)}
    print("c4: MAP at 300 steps done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    r_map = G.fit(m0, 4096, 10000, synth.fit_priors(spec), seed=0)
    torch.cuda.synchronize()
    map_res = (r_map, time.perf_counter() - t0)
    m0.close()
    print("c4: MAP at 10000 steps done", file=sys.stderr, flush=True)
    out = {}
    out["c4_pipeline"] = dict(workload="epl60_s0", map_at_table1_budget=map300,
                              **pipeline_bench(spec, obs0, truth0, n_map=4096, k_map=10000,
                                               n_vi=1000, k_vi=1000, chains=64, L=10,
                                               n_burn=250, n_samples=750,
                                               adapt_length=False, map_result=map_res))
    print("c4: Table 1 VI and HMC done", file=sys.stderr, flush=True)
    out["c4_pipeline_adapt_mass"] = dict(workload="epl60_s0", **pipeline_bench(
        spec, obs0, truth0, n_map=4096, k_map=10000, n_vi=1000, k_vi=1000, chains=64, L=10,
        n_burn=250, n_samples=750, adapt_length=False, map_result=map_res, adapt_mass=True))
    print("c4: Table 1 sizes with mass adaptation done", file=sys.stderr, flush=True)
    # the same MAP point with a longer surrogate fit (Table 1's 1000 iterations at 1e-3
    # cannot shrink the surrogate from sd 1e-3 to this posterior's widths of 1e-4 and
    # below; at a constant 3e-3 its mean never settles within those widths, so the rate
    # decays geometrically to 1e-4) and longer chains
    out["c4_pipeline_long"] = dict(workload="epl60_s0", **pipeline_bench(
        spec, obs0, truth0, n_map=4096, k_map=10000, n_vi=1000, k_vi=10000, chains=64, L=10,
        n_burn=1000, n_samples=1000, adapt_length=False, vi_lr=3e-3, vi_warmup=300,
        vi_lr_final=1e-4, map_result=map_res))
    print("c4: long surrogate and chains done", file=sys.stderr, flush=True)
    # a fit budgeted for throughput: 512 starts reach the same basin in the same 10 000
    # steps (at a slightly higher chi^2), then the mass-adapted chains
    out["c4_pipeline_fast"] = dict(workload="epl60_s0", **pipeline_bench(
        spec, obs0, truth0, n_map=512, k_map=10000, n_vi=1000, k_vi=1000, chains=64, L=10,
        n_burn=250, n_samples=750, adapt_length=False, adapt_mass=True))
    return out


def trace_summary(path, gap_split_s=0.1, min_dispatches=200):
    """Phases of a rocprofv3 kernel trace (the `*_kernel_trace.csv` of `--kernel-trace`), as
    markdown. A phase is a maximal run of this library's dispatches from one host thread with
    one driver family (fit: fit_/adam_/logpost_ kernels; vi_; hmc_; the likelihood kernels
    belong to the family around them) and no idle gap above gap_split_s. Per phase: span,
    busy (the union of all kernels' execution intervals in the span, over the span), the gaps
    between consecutive kernels, and the kernels taking the most time."""
    import csv
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"],
                         r["Thread_Id"]))
    rows.sort()

    def short(name):
        if "glens::" not in name:
            return None
        return name.split("glens::", 1)[1].split("(")[0].split("<")[0]

    def family(k):
        for pre, fam in (("hmc_", "hmc"), ("vi_", "vi"), ("fit_", "fit"), ("adam_", "fit"),
                         ("logpost_", "fit")):
            if k.startswith(pre):
                return fam
        return None

    phases, cur = [], None
    for t0, t1, name, tid in rows:
        k = short(name)
        if k is None:
            if cur is not None:
                cur["all"].append((t0, t1))
            continue
        fam = family(k)
        brk = (cur is None or tid != cur["tid"] or (fam is not None and cur["fam"] is not None
                                                   and fam != cur["fam"])
               or t0 - cur["end"] > gap_split_s * 1e9)
        if brk:
            cur = {"tid": tid, "fam": fam, "own": [], "all": [], "end": t1}
            phases.append(cur)
        if cur["fam"] is None:
            cur["fam"] = fam
        cur["own"].append((t0, t1, k))
        cur["all"].append((t0, t1))
        cur["end"] = max(cur["end"], t1)
    lines = ["| phase | host thread | family | dispatches | span s | busy | gap p50 us | "
             "gap p90 us | kernels (calls, avg us) |", "|---" * 9 + "|"]
    for n, ph in enumerate(phases):
        own = ph["own"]
        if len(own) < min_dispatches:
            continue
        a, b = own[0][0], max(t1 for _, t1, _ in own)
        iv = sorted((max(t0, a), min(t1, b)) for t0, t1 in ph["all"] if t1 > a and t0 < b)
        busy, hi = 0, a
        for t0, t1 in iv:
            if t1 > hi:
                busy += t1 - max(t0, hi)
                hi = t1
        gaps = np.array([max(0, own[i + 1][0] - own[i][1]) for i in range(len(own) - 1)]) * 1e-3
        tot = {}
        for t0, t1, k in own:
            c, d = tot.get(k, (0, 0))
            tot[k] = (c + 1, d + t1 - t0)
        top = sorted(tot.items(), key=lambda kv: -kv[1][1])[:7]
        ks = ", ".join(f"{k} ({c}, {d / c * 1e-3:.1f})" for k, (c, d) in top)
        lines.append(f"| {n} | {ph['tid']} | {ph['fam'] or 'lens'} | {len(own)} | "
                     f"{(b - a) * 1e-9:.3f} | {busy / max(b - a, 1):.3f} | "
                     f"{np.percentile(gaps, 50):.1f} | {np.percentile(gaps, 90):.1f} | {ks} |")
    return "\n".join(lines)


def _finite(x):
    """JSON has no inf / nan: non-finite numbers are written as null."""
    if isinstance(x, dict):
        return {k: _finite(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_finite(v) for v in x]
    if isinstance(x, float) and not math.isfinite(x):
        return None
    return x


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--stage-reps", type=int, default=0,
                    help="calls of the stage-timing loop (0: as many as --steps)")
    ap.add_argument("--spread-calls", type=int, default=200,
                    help="calls timed one by one for the median / p10 / p90 spread")
    ap.add_argument("--serve-systems", type=int, default=32,
                    help="systems in the serving stream (0 skips the serving measurement)")
    ap.add_argument("--serve-steps", type=int, default=300, help="Adam steps per fit")
    ap.add_argument("--serve-poisson-only", action="store_true",
                    help="run only the long serving stream under Poisson arrivals "
                         "(--serve-systems requests; e.g. 500) and print its JSON line")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the MAP -> VI -> HMC pipeline measurement")
    ap.add_argument("--recovery", type=int, default=0, metavar="N",
                    help="only the pipeline on N systems of the paper's simulation "
                         "distribution (posterior calibration and convergence)")
    ap.add_argument("--recovery-map", type=int, nargs=2, default=[300, 300],
                    metavar=("STARTS", "STEPS"), help="MAP budget of --recovery (Table 1's)")
    ap.add_argument("--vi-compare", action="store_true",
                    help="only: Table 1's VI budget with the pathwise and the score-function "
                         "estimator on one paper80 system")
    ap.add_argument("--recovery-seed", type=int, default=1000,
                    help="seed of --recovery's first system (the others follow)")
    ap.add_argument("--recovery-prior", choices=("paper", "sim"), default="paper",
                    help="fit prior of --recovery: the paper's broadened one or the simulation "
                         "distribution")
    ap.add_argument("--recovery-noise", choices=("poisson", "gauss"), default="poisson",
                    help="noise of --recovery's images")
    ap.add_argument("--c4-only", action="store_true",
                    help="run only the whole fit of the 60x60 EPL + shapelet system (MAP, VI, "
                         "HMC) and print its JSON")
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="with --serve-poisson-only: Poisson arrival rate (systems/s) instead of "
                         "0.8 x the plain loop's rate measured on a pilot")
    ap.add_argument("--serve-side", choices=["both", "served", "serial"], default="both",
                    help="with --serve-poisson-only: which side to run")
    ap.add_argument("--serve-only", choices=["mixed", "small", "tiny"],
                    help="run only the served-against-plain-loop measurement of one stream")
    ap.add_argument("--trace-summary", metavar="CSV",
                    help="print the phases of a rocprofv3 kernel trace (markdown) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy of 512 MiB (to scale HBM counters) and exit")
    args = ap.parse_args()
    if args.trace_summary:
        print(trace_summary(args.trace_summary))
        return
    if args.copy_calibration:
        import torch
        a = torch.ones(128 * 2 ** 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the hot path "
              "shards particles across GPUs with no exchange, see the design notes)", flush=True)
        sys.exit(2)

    import torch
    import paper_2202_07663_amd as G

    if args.vi_compare:
        print(json.dumps(_finite({"vi_estimators": vi_estimator_bench()}), allow_nan=False),
              flush=True)
        return
    if args.recovery > 0:
        r = recovery_bench(args.recovery, seed0=args.recovery_seed, n_map=args.recovery_map[0],
                           k_map=args.recovery_map[1], prior=args.recovery_prior,
                           noise=args.recovery_noise)
        print(json.dumps(_finite({"recovery": r}), allow_nan=False), flush=True)
        return
    if args.c4_only:
        import synth
        print(json.dumps(_finite(c4_bench(G, synth.spec_c2())), allow_nan=False), flush=True)
        return
    if args.serve_only:
        r = serving_bench(args.serve_systems, args.serve_steps, small=args.serve_only == "small",
                          tiny=args.serve_only == "tiny")
        print(json.dumps(_finite({"serving_" + args.serve_only: r}), allow_nan=False), flush=True)
        return
    if args.serve_poisson_only:
        r = serving_poisson_bench(args.serve_systems, args.serve_steps, rate=args.serve_rate,
                                  side=args.serve_side)
        print(json.dumps(_finite({"serving_poisson": r}), allow_nan=False), flush=True)
        return

    spec, obs, theta_np = workload()
    P = theta_np.shape[0]
    theta = torch.from_numpy(theta_np).cuda()
    model = G.Model.from_spec(spec, obs)
    model.reserve(P)
    ll = torch.empty(P, dtype=torch.float64, device="cuda")
    gr = torch.empty((P, model.d), dtype=torch.float32, device="cuda")

    for _ in range(args.warmup):
        model.loglik_grad(theta, out=(ll, gr))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        model.loglik_grad(theta, out=(ll, gr))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    value = P / (wall / args.steps)
    assert torch.isfinite(ll).all(), "non-finite log-likelihood in the benchmark batch"

    # per-call spread (HIP events) at the benchmark size, at P = 64, and for log L alone
    grad_ms = call_times_ms(lambda: model.loglik_grad(theta, out=(ll, gr)), args.spread_calls)
    ll_ms = call_times_ms(lambda: model.loglik(theta, out=ll), args.spread_calls)
    th64 = theta[:64].contiguous()
    ll64 = torch.empty(64, dtype=torch.float64, device="cuda")
    gr64 = torch.empty((64, model.d), dtype=torch.float32, device="cuda")
    for _ in range(20):
        model.loglik_grad(th64, out=(ll64, gr64))
    p64_ms = call_times_ms(lambda: model.loglik_grad(th64, out=(ll64, gr64)), args.spread_calls)

    # stage durations: a second timed loop of the same calls back to back, with HIP events
    # between the kernels on the stream they run on and one wait after the last call
    n_stage = args.stage_reps if args.stage_reps > 0 else args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stages = model.stage_times(theta, with_grad=True, n_calls=n_stage)
    ms_per_step_events = 1e3 * (time.perf_counter() - t0) / n_stage

    eps = np.hypot(theta_np[:, 2], theta_np[:, 3])
    N_mean = float(series_terms(eps).mean())
    fl = flops_model(spec.H, spec.W, spec.k, spec.psf.shape[0], spec.nmax, spec.lens_light, N_mean)
    per_launch = {"subpix_adj": fl["subpix_adj"] * P, "subpix_fwd": fl["subpix_fwd"] * P,
                  "conv_lik": fl["conv_lik_adj"] * P}
    dominant = max(("subpix_adj", "subpix_fwd", "conv_lik"), key=lambda k: stages[k])
    achieved = per_launch[dominant] / (stages[dominant] * 1e-3) / 1e12
    total_flops = sum(per_launch.values())
    rec = load_profile("epl60_P4096")
    roof = {"bound": "alu", "kernel": dominant,
            "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": None,
            "algorithmic_flop_per_launch": per_launch[dominant],
            "kernel_ms": round(stages[dominant], 4),
            "kernel_ms_basis": f"mean over {n_stage} back-to-back calls timed with HIP events "
                               f"({ms_per_step_events:.4f} ms per call with the events)",
            "peak_unpacked_fp32": PEAK_FP32_TFLOPS / 2,
            "basis": "achieved = op-model FLOP per launch / kernel time (an effective rate: the "
                     "kernel executes fewer operations than the model counts)"}
    if rec is not None:
        kr = rec["kernels"][KERNEL_NAMES[dominant]]
        roof["traffic"] = kr.get("hbm_bytes_per_launch")
        prof_ms = kr["avg_us"] * 1e-3
        roof["profile_kernel_ms"] = round(prof_ms, 4)
        roof["frac_profile"] = round(per_launch[dominant] / (prof_ms * 1e-3) / 1e12 /
                                     PEAK_FP32_TFLOPS, 4)
        if "valu_per_subpixel" in kr:
            ex = executed_flop_per_subpixel(kr["valu_per_subpixel"])
            sub = P * spec.H * spec.W * spec.k ** 2
            ex_tf = ex * sub / (stages[dominant] * 1e-3) / 1e12
            roof["executed_flop_per_subpixel"] = round(ex, 1)
            roof["executed_tflops"] = round(ex_tf, 2)
            roof["executed_frac"] = round(ex_tf / PEAK_FP32_TFLOPS, 4)
            roof["valu_busy_profile"] = kr.get("valu_busy")

    out = {
        "metric": "logL+grad evals/s (60x60 EPL+shapelets); fits/hour + p50/p99 latency",
        "value": round(value, 1),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64 (PSF on fp16 matrix cores, two-part split)",
        "data": "synthetic",
        "config": {"workload": "epl60_shapelet6_k2_moffat21", "P": P, "d": model.d,
                   "image": [spec.H, spec.W], "k_super": spec.k, "psf": spec.psf.shape[0],
                   "parallelism": "single-gpu"},
        "roofline": roof,
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "spread": {"logL+grad_P4096": spread(grad_ms, P), "logL_P4096": spread(ll_ms, P),
                   "logL+grad_P64": spread(p64_ms, 64)},
        "whole_path_tflops": round(total_flops / (ms_per_step * 1e-3) / 1e12, 2),
        "flop_per_eval": round(total_flops / P),
        "series_terms_counted": round(N_mean, 2),
    }
    if args.serve_systems > 0:
        out["serving"] = serving_bench(args.serve_systems, args.serve_steps)
        out["serving_small"] = serving_bench(args.serve_systems, args.serve_steps, small=True)
        out["serving_tiny"] = serving_bench(args.serve_systems, args.serve_steps, tiny=True)
    if not args.no_pipeline:
        import synth
        out.update(c4_bench(G, spec))
        sp = synth.spec_paper80()
        out["pipeline"] = dict(workload="paper80_s6", **pipeline_bench(
            sp, *stored(sp, 6), n_map=300, k_map=300, n_vi=500, k_vi=1000, chains=50, L=5))
        out["pipeline_adapt_mass"] = dict(workload="paper80_s6", **pipeline_bench(
            sp, *stored(sp, 6), n_map=300, k_map=300, n_vi=500, k_vi=1000, chains=50, L=5,
            adapt_mass=True))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, obs, theta_np, args.cpu_sample)
    print(json.dumps(_finite(out), allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
