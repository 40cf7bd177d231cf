"""Benchmark: ETRS steps/s of the non-collinear TDDFT step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload solid|cluster|large|grad|tiny|laser|kpoints]
                [--precision fp64|mixed] [--no-cpu-baseline] [--no-mixed] [--no-adjoint]
                [--no-ground-state] [--no-large] [--copy-probe]

Default: the solid-like system (64^3 grid, 256 two-component spinor states, 16 atoms x 18 KB+SOC
projectors on a jittered bcc lattice, circular B pulse, self-consistent exchange + Hartree,
dt = 0.05) in FP64, all inputs resident in HBM: exactly K timed ETRS steps after W untimed ones.
Its state set (2.1 GB) is far larger than the 256 MB Infinity Cache, so the passes stream from
HBM.  One JSON line follows, with

  roofline      the dominant kernel (the fused plane pass): algorithmic bytes per launch over its
                average duration, from HIP events on the stream it runs on (one launch in
                TIMING_STRIDE recorded), against 8 TB/s; `traffic` is the HBM bytes per launch from
                the committed rocprofv3 PMC summary while the kernel source is unchanged
  fp32_mixed    the same workload in the FP32-mixed form, with its own roofline
  large         the 96^3 x 512 spinor workload (32 atoms) in FP32-mixed: steps/s, its roofline
                and the adjoint/forward ratio of its recompute-mode adjoint step
  large_gradient  dM_z/dtheta of its 8 pulse parameters through PulseMz (checkpoint every 25
                steps in host memory, sub-segments of 5) over --large-gradient-steps steps:
                forward and backward wall time and peak device memory (--large-gradient-fd: one
                component against a fourth-order central difference)
  adjoint       adjoint/forward time ratio on the gradient workload (32^3 x 32, taped segments)
  ground_state  imaginary-time iterations/s of the headline workload
  cpu_baseline  the CPU oracle timed on this host (one ETRS step, scipy.fft on every core; and one
                H application on one core)
"""
import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TDDFT steps/s + Hψ HBM GB/s, FP64 vs FP32-mixed; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}
# In the timed region HIP events ride on one plane-pass launch in TIMING_STRIDE (coprime with the
# 12 plane passes of a step, so every stage position is sampled); each recorded launch costs the
# stream ~10 us.
TIMING_STRIDE = 5
GS_TAU = 0.02  # imaginary-time step: tau |H_max| ~ 1.7 at h = 0.42 bohr, inside T_4's stable range
XC_NAMES = {0: "none", 1: "Slater exchange, locally collinear",
            2: "Slater exchange + PW92 correlation (LSDA), locally collinear"}
ADJ_REPEATS = 3
WORKLOADS = {"tiny": 0, "cluster": 1, "solid": 2, "grad": 3, "large": 4, "laser": 5, "kpoints": 6}
PROFILE_KEYS = {0: "tiny16", 1: "cluster48", 2: "solid64", 3: "grad32", 4: "large96", 5: "laser48",
                6: "kpoints64"}
KERNEL_SOURCE = os.path.join(ROOT, "paper_2506_21908_amd", "csrc", "nct_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "plane_stage_solid64_fp64_traffic.md")
FFT_HEADER = os.path.join(ROOT, "paper_2506_21908_amd", "csrc", "nct_fft.hpp")
PLANE_BEGIN = "// ---------------------------------------------------------------- streamed global access"
PLANE_END = "// ---------------------------------------------------------------- plane pass: transform only"


def dataclass_dict(p) -> dict:
    return {k: (list(v) if isinstance(v, tuple) else v) for k, v in vars(p).items()}


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the plane-pass source (its streaming helpers, both plane-stage kernels and the FFT
    header they use): PMC traffic taken for it stays valid while this text is unchanged."""
    src = open(KERNEL_SOURCE).read()
    a, b = src.find(PLANE_BEGIN), src.find(PLANE_END)
    body = src[a:b] if 0 <= a < b else src
    h = hashlib.sha256(body.encode())
    h.update(open(FFT_HEADER, "rb").read())
    return h.hexdigest()[:16]


def traffic_path(key: str, precision: str) -> str:
    return os.path.join(PROFILES, f"plane_stage_{key}_{precision}_traffic.md")


def read_traffic(precision: str, path: str = None):
    """HBM bytes per plane-pass launch from a committed rocprofv3 PMC summary (by default the
    headline workload's, FP64 or FP32-mixed), if the kernel source is unchanged since the
    counters were taken; else None."""
    if path is None:
        path = TRAFFIC_FILE if precision == "fp64" else TRAFFIC_FILE.replace("fp64", "mixed")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("traffic:"):
            for kv in line.split()[1:]:
                k, v = kv.split("=")
                vals[k] = v
    if vals.get("kernel_sha") != kernel_hash():
        return None
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_info():
    """Host CPU model, the cores this process may use, and the BLAS thread count."""
    model = platform.processor() or ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    blas = None
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        blas = [{"api": d.get("internal_api"), "threads": d.get("num_threads")} for d in info
                if d.get("user_api") == "blas"]
    except Exception:  # threadpoolctl missing or failing: report nothing rather than guess
        blas = None
    return {"cpu_model": model, "cores": len(os.sched_getaffinity(0)), "blas": blas}


def cpu_baseline(w, budget_s: float = 45.0):
    """The oracle, as it stands, on this host's cores: ETRS steps of the workload with scipy.fft on
    every core (at least one, more while the budget allows), then one H application of the whole
    state set with scipy.fft on one core."""
    from oracle import nct_oracle as O
    info = host_info()
    cores = info["cores"]
    O.FFT_WORKERS = cores
    sysd = O.system_from_workload(w)
    t0 = time.perf_counter()
    psi = O.etrs_step(sysd, w.psi0, 0.0)
    el = time.perf_counter() - t0
    n = 1
    while time.perf_counter() - t0 + el < budget_s and n < 3:
        psi = O.etrs_step(sysd, psi, n * w.dt)
        n += 1
    el = time.perf_counter() - t0
    out = {"value": n / el, "unit": "steps/s", "cores": cores, "kind": "oracle",
           "sample": f"{n} ETRS step(s) of the {w.name} workload (numpy/scipy FP64, "
                     f"scipy.fft workers={cores}), {el:.1f} s", "host": info}
    del psi
    O.FFT_WORKERS = 1
    F = O.fields_from_density(sysd, O.spin_density(w.psi0, sysd.occ), 0.0)
    t1 = time.perf_counter()
    O.apply_hamiltonian(sysd, w.psi0, F)
    h1 = time.perf_counter() - t1
    O.FFT_WORKERS = -1
    out["one_core"] = {"H_application_s": h1, "cores": 1,
                       "sample": f"one H application of all {w.nstates} states of the {w.name} "
                                 f"workload, scipy.fft workers=1 (an ETRS step makes 12)"}
    return out


def large_gradient(wl, nsteps, checkpoint_every, sub_every, fd):
    """dM_z(T)/dtheta of the 8 pulse parameters on the large workload in FP32-mixed through
    PulseMz with the two-level recompute schedule (checkpoints in host memory), timed; with fd,
    one parameter (the largest component) against a fourth-order central difference of the same
    trajectory."""
    import numpy as np
    import torch
    from paper_2506_21908_amd import nct
    pf = nct.NCT_FP32_MIXED
    s = nct.system_from_workload(wl, precision=pf)
    psi0 = nct.states_to_device(wl.psi0, pf)
    pulses = wl.bfield.pulses
    th0 = np.array([p.A for p in pulses] + [p.omega for p in pulses])
    theta = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    peak = [0.0]

    def used():
        f, t = torch.cuda.mem_get_info()
        return (t - f) / 1e9

    def prog(k, n):
        peak[0] = max(peak[0], used())
        say(f"large gradient: backward segment {k}/{n}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L = nct.pulse_mz(theta, s, psi0, pulses, nsteps, checkpoint_every, checkpoint_on_host=True,
                     sub_every=sub_every, progress=prog)
    torch.cuda.synchronize()
    t_f = time.perf_counter() - t0
    peak[0] = max(peak[0], used())
    say(f"large gradient: {nsteps}-step forward in {t_f:.1f} s")
    t0 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    g = theta.grad.numpy().copy()
    out = {"workload": wl.name, "precision": "mixed", "steps": nsteps,
           "checkpoint_every": checkpoint_every, "sub_every": sub_every,
           "checkpoints": "host memory", "L_Mz": float(L.detach()),
           "forward_s": t_f, "backward_s": t_b, "ratio": t_b / t_f,
           "device_used_GB_peak": peak[0], "gradient": g.tolist(),
           "definition": "backward wall time (segment and sub-segment re-runs, recompute-mode "
                         "backward steps) / forward wall time of the same trajectory"}
    if fd:
        k = int(np.argmax(np.abs(g)))
        h = 0.05 * abs(th0[k])

        def L_at(dk):
            th = th0.copy()
            th[k] += dk
            s.set_potentials(B0=(0.0, 0.0, 0.0), pulses=nct._pulses_with(pulses, th))
            psi = psi0.clone()
            s.step(psi, 0.0, nsteps)
            tot = s.density_magnetization(psi, nsteps * wl.dt, totals=True)
            say(f"large gradient: L at theta_{k} {dk:+.3e}: {tot[3]:.10f}")
            return float(tot[3])

        Lp1, Lm1, Lp2, Lm2 = L_at(h), L_at(-h), L_at(2 * h), L_at(-2 * h)
        fd4 = (8.0 * (Lp1 - Lm1) - (Lp2 - Lm2)) / (12.0 * h)
        out["fd_check"] = {"parameter": k, "h": h, "adjoint": float(g[k]), "central_difference_4th": fd4,
                           "rel_diff": abs(g[k] - fd4) / abs(fd4)}
    s.close()
    del psi0
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="solid", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--xc", type=int, default=None, choices=[0, 1, 2],
                    help="override the workload's exchange-correlation (2: + PW92 correlation)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32-mixed run of the workload")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward ratios")
    ap.add_argument("--adjoint-segment", type=int, default=20)
    ap.add_argument("--no-ground-state", action="store_true", help="skip the ground-state timing")
    ap.add_argument("--no-large", action="store_true", help="skip the 96^3 x 512 FP32-mixed entry")
    ap.add_argument("--large-steps", type=int, default=10)
    ap.add_argument("--large-gradient-steps", type=int, default=50,
                    help="trajectory length of the large-workload pulse gradient (0: skip)")
    ap.add_argument("--large-gradient-fd", action="store_true",
                    help="check one gradient component against central differences")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain 1 GiB device copy first (PMC scale reference)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only (a state-sharded multi-GPU path is not "
              "implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2506_21908_amd import inputs as I
    from paper_2506_21908_amd import nct

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t_start = time.perf_counter()
    case = WORKLOADS[args.workload]
    w = I.workload(case)
    if args.xc is not None:
        w.xc = args.xc
    say(f"workload {w.name} built in {time.perf_counter() - t_start:.1f} s")

    if args.copy_probe:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def run(wl, precision_flag, steps, warmup, breakdown_steps=0):
        """Timed region: exactly `steps` ETRS steps; HIP events only on the plane pass (one launch
        in TIMING_STRIDE).  Then, outside the timed region, `breakdown_steps` more steps with
        every kernel class instrumented for the per-kernel breakdown."""
        s = nct.system_from_workload(wl, precision=precision_flag)
        psi = nct.states_to_device(wl.psi0, precision_flag)
        t = 0.0
        if warmup:
            s.step(psi, t, warmup)
            t += warmup * wl.dt
        torch.cuda.synchronize()
        s.set_timing_sample(TIMING_STRIDE)
        s.set_timing(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(psi, t, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        tim = s.timing()
        full = None
        if breakdown_steps:
            s.set_timing_sample(1)
            s.set_timing(-1)
            s.step(psi, t + steps * wl.dt, breakdown_steps)
            full = s.timing()
        s.close()
        del psi
        torch.cuda.empty_cache()
        return el, tim, full

    def roofline(tim, key, prec):
        ms, cnt, by, _ = tim["plane_stage"]
        achieved = (by / cnt) / (ms / cnt * 1e-3) / 1e9 if cnt else 0.0
        return {"kernel": "k_plane_stage (fused plane pass)", "bound": "hbm",
                "timed_launches": cnt, "timing_stride": TIMING_STRIDE,
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": read_traffic(prec, traffic_path(key, prec)),
                "algorithmic_bytes_per_launch": by / cnt if cnt else None,
                "avg_launch_ms": ms / cnt if cnt else None}

    def breakdown(full, nb, prec):
        hp_ms = sum(full[k][0] for k in ("plane_stage", "xpass", "proj"))
        hp_by = sum(full[k][2] for k in ("plane_stage", "xpass", "proj"))
        xs, pj = full["xpass"], full["proj"]
        peak = MFMA_PEAK_TFLOPS[prec]
        proj = None
        if pj[0] > 0:
            tf = pj[3] / (pj[0] * 1e-3) / 1e12          # useful flops (P projectors per atom)
            ai = pj[3] / pj[2] if pj[2] > 0 else None    # flop per algorithmic byte
            bound = min(peak, ai * HBM_PEAK_GBS / 1e3) if ai else peak
            proj = {"useful_TFLOPs": tf, "peak_TFLOPs": peak, "frac_of_peak": tf / peak,
                    "flop_per_byte": ai, "ai_x_bw_bound_TFLOPs": bound, "frac_of_bound": tf / bound,
                    "ms_per_step": pj[0] / nb, "launches_per_step": pj[1] / nb,
                    "flops_definition": "8 flop per complex multiply-add over the method's "
                                        "projectors per atom (18), contraction and scatter"}
        return {
            "hpsi_GBps": hp_by / (hp_ms * 1e-3) / 1e9 if hp_ms > 0 else None,
            "xpass_GBps": xs[2] / (xs[0] * 1e-3) / 1e9 if xs[0] > 0 else None,
            "projector_mfma": proj,
            "kernel_breakdown": {k: {"ms_per_step": v[0] / nb, "launches_per_step": v[1] / nb,
                                     "GBps": (v[2] / (v[0] * 1e-3) / 1e9) if v[0] > 0 else None}
                                 for k, v in full.items() if v[1] > 0},
            "kernel_breakdown_note": f"separate {nb}-step pass with every kernel class instrumented",
        }

    key = PROFILE_KEYS[case]
    pflag = nct.NCT_FP64 if args.precision == "fp64" else nct.NCT_FP32_MIXED
    nb = 10
    el, tim, full = run(w, pflag, args.steps, args.warmup, breakdown_steps=nb)
    say(f"{args.steps} steps in {el:.3f} s")
    value = args.steps / el

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.n), "cell_bohr": w.L[0],
                   "spinor_states": w.nstates, "atoms": w.natoms,
                   "projectors_per_atom": sum(c.twoj + 1 for c in w.channels),
                   "dt": w.dt, "taylor_order": w.taylor_order, "propagator": "ETRS",
                   "xc": XC_NAMES[w.xc], "hartree": "FFT",
                   "b_pulses": [dataclass_dict(p) for p in w.bfield.pulses] or None,
                   "laser": [dataclass_dict(p) for p in w.laser] or None,
                   "precision": args.precision, "parallelism": "single GPU",
                   "psi_GB": 2 * w.nstates * w.npoints * (16 if args.precision == "fp64" else 8) / 1e9},
        "roofline": roofline(tim, key, args.precision),
    }
    out.update(breakdown(full, nb, args.precision))

    if not args.no_mixed and args.precision == "fp64":
        el2, tim2, full2 = run(w, nct.NCT_FP32_MIXED, args.steps, args.warmup, breakdown_steps=nb)
        say(f"FP32-mixed: {args.steps} steps in {el2:.3f} s")
        out["fp32_mixed"] = {"value": args.steps / el2, "unit": "steps/s",
                             "ms_per_step": 1e3 * el2 / args.steps, "dtype": "f32+f64",
                             "roofline": roofline(tim2, key, "mixed"),
                             "xpass_GBps": breakdown(full2, nb, "mixed")["xpass_GBps"],
                             "projector_mfma": breakdown(full2, nb, "mixed")["projector_mfma"]}

    if not args.no_ground_state and w.natoms > 0 and w.xc <= 2:
        # ground state by imaginary time from the initial spin-density matrix (10 iterations)
        s = nct.system_from_workload(w, precision=pflag)
        dens = I.atom_densities(w)
        psi = nct.states_to_device(w.psi0, pflag)
        s.dm_initialization(dens, update_fields=True)
        s.ground_state(psi.clone(), 1, GS_TAU, keep_fields=True)   # untimed: allocates its buffers
        s.dm_initialization(dens, update_fields=True)
        torch.cuda.synchronize()
        s.set_timing(1 << 8)   # the orthonormalisation class only
        t0 = time.perf_counter()
        E = s.ground_state(psi, 10, GS_TAU, keep_fields=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        oms, ocnt, oby, ofl = s.timing()["orth"]
        out["ground_state"] = {"iterations_per_s": 10 / el, "tau": GS_TAU,
                               "energy_first": float(E[0]), "energy_last": float(E[-1]),
                               "orthonormalisation_ms_per_iteration": oms / 10,
                               "orthonormalisation_TFLOPs": (ofl / (oms * 1e-3) / 1e12) if oms > 0 else None,
                               "definition": "imaginary-time iteration: T_K(-tau H) on all states, "
                                             "orthonormalisation (overlap and change of basis on "
                                             "the matrix cores, FP64 accumulation; S x S Cholesky "
                                             "on the host), density and fields"}
        s.close()
        del psi
        torch.cuda.empty_cache()
        say("ground state timed")

    if not args.no_adjoint:
        # taped segments on the gradient workload (32^3 x 32, 2 atoms, 4 pulses): the tape of a
        # segment holds 3K state sets per step
        wg = I.workload(3)
        C = args.adjoint_segment
        s = nct.system_from_workload(wg, precision=nct.NCT_FP64, tape_steps=C)
        lam = torch.empty_like(nct.states_to_device(wg.psi0))
        # a segment takes ~20 ms, so each time is the minimum over ADJ_REPEATS repeats (the
        # first backward pass of a process also pays one-off host costs)
        t_fwd = t_tape = t_bwd = float("inf")
        for _ in range(ADJ_REPEATS):
            psi = nct.states_to_device(wg.psi0)
            s.step(psi, 0.0, 2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(psi, 0.1, C)
            torch.cuda.synchronize()
            t_fwd = min(t_fwd, time.perf_counter() - t0)
            s.magnetization_seed(psi, (0.0, 0.0, 1.0), lam)
            psi_c = nct.states_to_device(wg.psi0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(psi_c, 0.0, C, tape=True)
            torch.cuda.synchronize()
            t_tape = min(t_tape, time.perf_counter() - t0)
            for j in reversed(range(C)):
                s.backward_step(j, None, j * wg.dt, lam, lam)
            torch.cuda.synchronize()
            t_bwd = min(t_bwd, time.perf_counter() - t0)
        out["adjoint"] = {"workload": wg.name, "precision": "fp64", "ratio": t_bwd / t_fwd,
                          "segment_steps": C, "repeats": ADJ_REPEATS, "statistic": "minimum over repeats",
                          "forward_ms_per_step": 1e3 * t_fwd / C,
                          "taped_forward_ms_per_step": 1e3 * t_tape / C,
                          "backward_ms_per_step_incl_taped_rerun": 1e3 * t_bwd / C,
                          "ratio_without_rerun": (t_bwd - t_tape) / t_fwd,
                          "definition": "(taped re-run of the segment + backward steps) / forward steps"}
        s.close()
        del psi, psi_c, lam
        torch.cuda.empty_cache()
        say("adjoint timed")

    if not args.no_large and case != 4:
        t0 = time.perf_counter()
        wl = I.workload(4)
        say(f"workload {wl.name} built in {time.perf_counter() - t0:.1f} s")
        K = args.large_steps
        el3, tim3, _ = run(wl, nct.NCT_FP32_MIXED, K, 2)
        say(f"large FP32-mixed: {K} steps in {el3:.3f} s")
        large = {"workload": wl.name, "grid": list(wl.n), "spinor_states": wl.nstates,
                 "atoms": wl.natoms, "precision": "mixed", "dtype": "f32+f64", "steps": K,
                 "value": K / el3, "unit": "steps/s", "ms_per_step": 1e3 * el3 / K,
                 "psi_GB": 2 * wl.nstates * wl.npoints * 8 / 1e9,
                 "roofline": roofline(tim3, "large96", "mixed")}
        if not args.no_adjoint:
            # recompute-mode adjoint step: the step is re-run from psi_n with a one-step tape
            s = nct.system_from_workload(wl, precision=nct.NCT_FP32_MIXED)
            psi = nct.states_to_device(wl.psi0, nct.NCT_FP32_MIXED)
            lam = torch.empty_like(psi)
            s.step(psi, 0.0, 1)
            s.magnetization_seed(psi, (0.0, 0.0, 1.0), lam)
            psi_n = psi.clone()
            s.backward_step(-1, psi_n, 0.05, lam, lam)     # untimed: allocates the one-step tape
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(psi, 0.05, 2)
            torch.cuda.synchronize()
            t_f = (time.perf_counter() - t0) / 2
            t0 = time.perf_counter()
            for _ in range(2):
                s.backward_step(-1, psi_n, 0.05, lam, lam)
            torch.cuda.synchronize()
            t_b = (time.perf_counter() - t0) / 2
            large["adjoint"] = {"ratio": t_b / t_f, "forward_ms_per_step": 1e3 * t_f,
                                "backward_ms_per_step": 1e3 * t_b,
                                "device_used_GB": (lambda f: (f[1] - f[0]) / 1e9)(torch.cuda.mem_get_info()),
                                "definition": "recompute-mode backward_step (the forward step "
                                              "re-run from psi_n with its tape, then the reverse "
                                              "step) / forward step"}
            s.close()
            del psi, psi_n, lam
            torch.cuda.empty_cache()
        out["large"] = large
        if args.large_gradient_steps > 0:
            out["large_gradient"] = large_gradient(wl, args.large_gradient_steps, 25, 5,
                                                   args.large_gradient_fd)
        del wl
    elif case == 4 and args.large_gradient_steps > 0:
        out["large_gradient"] = large_gradient(w, args.large_gradient_steps, 25, 5, args.large_gradient_fd)

    if not args.no_cpu_baseline:
        say("timing the oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(w)
    out["bench_wall_s"] = time.perf_counter() - t_start
    print(json.dumps(out))


if __name__ == "__main__":
    main()
