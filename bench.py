#!/usr/bin/env python3
"""Benchmark: GSM solves/sec to a 1e-9 relative residual at 31^3 orders.

Workload (one step): the two bodies at M = 15 (31^3 harmonics, 64^3 FFT
grid) -- the cubic sphere lattice (Lambda = 0.3 lambda, r = 0.3 Lambda,
eps 4 in vacuum, 64^3 voxels) and the layered stack (fill 0.4, eps 2.25 / 9)
-- each driven by two orthogonal transverse polarisations along normal
incidence (z) plus D seeded incidence directions (default D = 31), all
directions of a body in one batched call; complex64 GMRES(30) inside FP64
iterative refinement to a relative FP64 residual of 1e-9.  That is
2 x 2 x (D + 1) = 128 solves per step, and each batched matrix-vector
product moves more than 1 GB, well beyond the 256 MB Infinity Cache.  The
literal 4-solve case (D = 0: x and y drives at normal incidence only) is
timed as well and reported as "as_configured".

Prints one JSON line: value = solves/s over the timed steps; the roofline of
the dominant kernel class (found in one extra profiled step before the timed
ones): its algorithmic bytes or flops over the durations of its launches in
the timed steps, one launch in four bracketed by a hipEvent pair on its own
stream (only that class carries events there); the per-class table of the
extra step; the whole step against HBM (the algorithmic bytes of all its
launches over its wall time); the plain FP64 GPU solve of the same workload; the literal 4-solve case, the
uneven 256-instance sweep, the 32^3-voxel inverse-design gradient and the
M = 31 woodpile batch as further lines of the same JSON object; Table 1's
single-solve workload at three sizes (context beside the paper's times); the
achievable copy bandwidth; the pole search of Eqs.(6)-(10) on the paper's
Fig. 2 lattices (E and H systems, beside the printed indices); the headline
batch through the H-field system of Eq.(5); the Fresnel-tensor retrieval on
Fig. 4's uniaxial lattices; and the CPU oracle (scipy.fft on the host
threads + SciPy GMRES, FP64) timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import resource
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# vector peaks of the chip as these kernels are built (packed FP32 off):
# 256 CUs x 64 lanes x 2 flop (one FMA per lane and clock) x 2.4 GHz, for
# FP32 and FP64 alike; the published FP32 figure (157.3) counts packed FMAs
ALU_UNPACKED_TFLOPS = {"c64": 78.6, "c128": 78.6}
# the transforms are additions and multiplications that do not fuse into
# FMAs: one flop per lane and clock, 256 x 64 x 2.4 GHz
ALU_ADD_ISSUE_TFLOPS = 39.3
TOL = 1e-9
CPU_SAMPLE_S = 10.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--directions", type=int, default=31,
                    help="seeded incidence directions per body besides normal incidence (batched)")
    ap.add_argument("--config-steps", type=int, default=5, help="steps of the 4-solve case")
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--sweep-steps", type=int, default=4,
                    help="steps of the uneven 256-instance sweep (0 skips it)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--design-steps", type=int, default=2,
                    help="timed gradients of the 32^3-voxel inverse-design case (0: skip)")
    ap.add_argument("--woodpile-steps", type=int, default=2,
                    help="timed batched calls of the M = 31 woodpile case (0: skip)")
    ap.add_argument("--group-max", type=int, default=None,
                    help="systems per launch group (default: the library's, 32; 0: one group per call)")
    ap.add_argument("--one-group-steps", type=int, default=None,
                    help="timed steps with one launch group per call, for the dominant kernel's own rate "
                         "(default: --steps; 0: skip)")
    ap.add_argument("--pole-steps", type=int, default=2,
                    help="timed rounds of the Fig. 2 pole searches (E and H systems, 0: skip)")
    ap.add_argument("--fresnel-steps", type=int, default=2,
                    help="timed rounds of the Fig. 4 Fresnel-tensor retrievals (0: skip)")
    ap.add_argument("--hfield-steps", type=int, default=2,
                    help="timed steps of the headline batch through the H-field system (0: skip)")
    ap.add_argument("--table1-reps", type=int, default=10,
                    help="timed single solves per size and precision of Table 1's workload (0: skip)")
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="residual reduction asked of each complex64 Krylov cycle (library default if unset)")
    ap.add_argument("--concurrent-bodies", action="store_true",
                    help="solve the two bodies of a step concurrently, one host thread and stream each "
                         "(with launch groups of 32 about 4%% more solves/s than one after the other; the "
                         "launches of the streams share the GPU, so the timed launch durations of the "
                         "roofline include the other streams' work and drift further from the profiler's "
                         "kernel durations); default: one after the other")
    ap.add_argument("--no-autotune", action="store_true",
                    help="fixed codelet families instead of timing them at the first solve")
    ap.add_argument("--matvec-systems", type=int, default=0,
                    help="with --matvec-only: apply the operator to the first N systems of the body (0: all)")
    ap.add_argument("--matvec-only", type=int, default=0, metavar="REPS",
                    help="for hardware-counter runs: a 1 GiB device copy (calibration), then REPS "
                         "batched operator applications of one body of the step in complex64 and "
                         "REPS in complex128; prints their wall times and exits")
    ap.add_argument("--profile", choices=("dominant", "all"), default="dominant",
                    help="kernel classes whose launches carry hipEvent pairs in the timed steps: "
                         "only the dominant one (found in one extra profiled step before them), "
                         "or all of them")
    ap.add_argument("--profile-every", type=int, default=4, metavar="K",
                    help="time one launch in K of each profiled class in the timed steps "
                         "(event pairs on every launch cost about 2%% of throughput)")
    return ap.parse_args()


def build_workload(gsm, inputs, directions, autotune=False):
    bodies = [inputs.sphere_lattice_m15(), inputs.layered_stack_m15()]
    work = []
    for w in bodies:
        lam, M = w["wavelength"], w["M"]
        k0 = 2 * np.pi / lam
        plan = gsm.Plan(w["eps"], w["period"], M, autotune=autotune)
        insts = []
        dirs = [np.array([0.0, 0.0, 1.0])]
        if directions:
            dirs += list(inputs.random_directions(directions, seed=7))
        for khat in dirs:
            a1 = inputs.transverse_drive(khat)
            a2 = np.cross(khat, a1)
            if np.allclose(khat, [0, 0, 1]):
                a1, a2 = np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
            inst = gsm.make_instance(lam, k0 * khat, M, [tuple(a1), tuple(a2)])
            inst.eps_b = plan.basis_eps(inst)
            insts.append(inst)
        work.append((plan, insts))
    return work


STATS = {"iterations": 0, "refinements": 0, "reorth": 0, "solves": 0}


class Bodies:
    """Runs the bodies of a step (one plan each) from one host thread per
    body, each on a stream of its own, so their launches interleave on the
    GPU; serial=True solves them one after the other instead."""

    def __init__(self, work, serial=False):
        import torch
        from concurrent.futures import ThreadPoolExecutor
        self.work = work
        self.serial = serial
        self.streams = [torch.cuda.Stream() for _ in work]
        self.pool = None if serial else ThreadPoolExecutor(len(work))

    def _one(self, i, opts):
        import torch
        plan, insts = self.work[i]
        s = self.streams[i]
        with torch.cuda.stream(s):
            return plan.solve(insts, opts, stream=s.cuda_stream)

    def solve(self, opts):
        if self.serial:
            return [self._one(i, opts) for i in range(len(self.work))]
        futs = [self.pool.submit(self._one, i, opts) for i in range(len(self.work))]
        return [f.result() for f in futs]


def run_step(gsm, bodies, opts):
    nsolve = 0
    worst = 0.0
    for E, info, st in bodies.solve(opts):
        if st != gsm.GSM_OK:
            raise RuntimeError(f"solve status {st}: {info}")
        nsolve += len(info)
        worst = max(worst, max(i["rel_residual"] for i in info))
        for i in info:
            for k in ("iterations", "refinements", "reorth"):
                STATS[k] += i[k]
        STATS["solves"] += len(info)
    return nsolve, worst


def uneven_sweep(gsm, inputs, steps, autotune):
    """256 (omega, k) points of an orthorhombic ellipsoid lattice (1 : 0.8 :
    1.2, semi-axes 0.35 / 0.25 / 0.15, eps 6, 64^3 voxels) with order counts
    drawn from 6..16 per point, one drive each: one call, its eleven (M, P)
    groups scheduled by the library; complex64 + FP64 refinement to 1e-9."""
    import torch
    lam, khat, Ms = inputs.orthorhombic_sweep()
    period = (1.0, 0.8, 1.2)
    eps = inputs.ellipsoid((64, 64, 64), period, (0.35, 0.25, 0.15), 6.0)
    plan = gsm.Plan(eps, period, (16, 16, 16), autotune=autotune)
    insts = []
    for i in range(lam.size):
        k = 2 * np.pi / lam[i] * khat[i]
        inst = gsm.make_instance(lam[i], k, (int(Ms[i]),) * 3, [tuple(inputs.transverse_drive(khat[i]))])
        inst.eps_b = plan.basis_eps(inst)
        insts.append(inst)
    opts = gsm.default_opts(tol=TOL, precision=gsm.GSM_MIXED, restart=30)
    # two untimed calls (the first tunes the codelet families and builds the
    # grids), then the timed ones
    for _ in range(2):
        plan.solve(insts, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, info, st = plan.solve(insts, opts)
        if st != gsm.GSM_OK:
            raise RuntimeError(f"sweep status {st}")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # one more call with every launch timed: the batched product's HBM rate
    gsm.profile_begin()
    plan.solve(insts, opts)
    prof = gsm.profile_end()
    families = {int(m): plan.tuning((int(m),) * 3)[0] for m in sorted(set(Ms.tolist()))}
    return {"value": round(len(insts) / dt, 3), "unit": "solves/s", "instances": len(insts),
            "order_counts": [int(Ms.min()), int(Ms.max())], "ms_per_step": round(dt * 1e3, 3),
            "codelet_families": families,
            "max_rel_residual": max(i["rel_residual"] for i in info),
            "fft_sizes": sorted({int(i["fft_size"]) for i in info}),
            "roofline": matvec_hbm(prof), "roofline_fp64_residual": matvec_hbm(prof, "c128")}


def cpu_baseline(inputs):
    """The oracle's FFT + GMRES route (FP64) on the normal-incidence solves of
    the step (sphere lattice and layered stack at M = 15, x and y drives, the
    same 1e-9 residual), taken in turn until about CPU_SAMPLE_S seconds have
    passed."""
    from oracle import gsm as O
    cases = []
    for w in (inputs.sphere_lattice_m15(), inputs.layered_stack_m15()):
        lam, M = w["wavelength"], w["M"]
        k = 2 * np.pi / lam * np.array([0.0, 0.0, 1.0])
        c = O.box_image(w["eps"], tuple(2 * m for m in M))
        q = O.harmonic_q(k, lam, w["period"], M)
        eb = float(np.mean(w["eps"]))
        for a in ((1.0, 0, 0), (0, 1.0, 0)):
            cases.append((c, M, q, eb, np.array(a, complex)))
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    n = its = 0
    while n == 0 or time.perf_counter() - t0 < CPU_SAMPLE_S:
        c, M, q, eb, a = cases[n % len(cases)]
        _, it = O.solve_fft_gmres(c, M, q, eb, a, (64, 64, 64), rtol=TOL)
        n += 1
        its += it
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    host = host_cpu()
    return {"value": n / wall, "unit": "solves/s", "cores": O.FFT_WORKERS,
            "cpu_time_over_wall": round(cpu / wall, 2), "host": host,
            "fft": f"scipy.fft, workers = {O.FFT_WORKERS} (OMP_NUM_THREADS, else the CPU affinity)",
            "kind": "oracle",
            "sample": f"{n} normal-incidence solves (sphere lattice and layered stack, M=15, x/y drives, "
                      f"FP64 scipy.fft (all host threads) + scipy GMRES(30) to 1e-9), {its} iterations, "
                      f"{wall:.1f} s wall"}


def matvec_only(gsm, body, reps, systems=0):
    """Copy calibration and bare operator applications (no solve), of the
    first `systems` systems of the body (0: all)."""
    import torch
    plan, insts = body
    if systems > 0:
        sizes = [len(gsm.system_sizes([i])) for i in insts]
        keep = int(np.searchsorted(np.cumsum(sizes), systems)) + 1
        insts = insts[:keep]
        if len(gsm.system_sizes(insts)) != systems:
            raise ValueError(f"no instance prefix of the body holds exactly {systems} systems")
    out = {}
    # a plain shader copy of 1 GiB (read 1 GiB, write 1 GiB): torch's
    # elementwise negation of 2^28 float32 values
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    out["copy_1GiB_ms"] = round((time.perf_counter() - t0) / 3 * 1e3, 3)
    del src, dst
    n = sum(gsm.system_sizes(insts))
    g = torch.Generator(device="cpu").manual_seed(11)
    for prec, dt, tag in ((gsm.GSM_MIXED, torch.complex64, "c64"), (gsm.GSM_FP64, torch.complex128, "c128")):
        x = torch.randn(n, dtype=dt, generator=g).to("cuda")
        plan.apply(insts, x, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.apply(insts, x, precision=prec)
        torch.cuda.synchronize()
        out[f"apply_{tag}_ms"] = round((time.perf_counter() - t0) / reps * 1e3, 3)
    out["systems"] = len(gsm.system_sizes(insts))
    print(json.dumps(out))


def roofline_of(name, v):
    """Roofline entry of one kernel class against the HBM bound: algorithmic
    bytes of its launches over their summed durations, against the 8 TB/s
    peak.  The vector-ALU side rides along: its algorithmic flops against the
    unpacked FMA rate and against the issue rate of plain additions and
    multiplications (what the transforms are made of)."""
    sec = v["ms"] * 1e-3
    gbs = v["bytes"] / sec / 1e9 if sec > 0 else 0.0
    tfs = v.get("flops", 0.0) / sec / 1e12 if sec > 0 else 0.0
    prec = "c128" if name.endswith("c128") else "c64"
    out = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": name,
           "avg_launch_us": round(v["ms"] * 1e3 / max(1, v["launches"]), 2), "timed_launches": v["launches"]}
    if v.get("flops", 0.0) > 0:
        out["alu"] = {"achieved": round(tfs, 2), "unit": "TFLOP/s",
                      "intensity_flop_per_byte": round(v["flops"] / max(v["bytes"], 1.0), 2),
                      "peak_fma": ALU_UNPACKED_TFLOPS[prec], "frac_fma": round(tfs / ALU_UNPACKED_TFLOPS[prec], 4),
                      "peak_add_issue": ALU_ADD_ISSUE_TFLOPS,
                      "frac_add_issue": round(tfs / ALU_ADD_ISSUE_TFLOPS, 4)}
    return out


def counted_traffic(name, systems=64):
    """HBM bytes per launch of kernel class `name` over `systems` systems from
    the committed hardware-counter record (FETCH_SIZE / WRITE_SIZE scaled by a
    copy-kernel calibration), or None when there is none or the kernel
    sources changed since it was taken."""
    tag = "" if systems == 64 else f"_{systems}sys"
    path = os.path.join(ROOT, "profiles", f"{name}_m15{tag}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec


def kernel_table(prof):
    return {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                "GBps": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None,
                "TFLOPs": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2) if v["ms"] > 0 and v["flops"] else None}
            for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}


def inverse_design(gsm, inputs, steps):
    """Gradient of ||eps_eff - diag(4, 5, 6)||_F^2 with respect to the 32^3
    voxel permittivities (Gaussian-smoothed seeded field stretched to
    [1, 10], Lambda = 0.3 lambda, M = 12, normal incidence) through the
    autograd function, as an optimisation loop would take it: each step
    builds the plan of the current voxels, solves the three drives (forward)
    and the three adjoint systems (backward), complex64 + FP64 refinement."""
    import torch
    eps0 = torch.tensor(inputs.smooth_random_field(32, seed=4), dtype=torch.float64, device="cuda:0")
    lam, M = 1 / 0.3, (12, 12, 12)
    inst = gsm.make_instance(lam, (0.0, 0.0, 2 * np.pi / lam), M)
    target = torch.diag(torch.tensor([4.0, 5.0, 6.0], dtype=torch.complex128, device="cuda:0"))
    fn = gsm.eff_tensor_fn()
    opts = gsm.default_opts(tol=TOL)

    def one():
        e = eps0.clone().requires_grad_(True)
        ee = fn.apply(e, (1.0, 1.0, 1.0), M, [inst], opts)
        ((ee[0] - target).abs() ** 2).sum().backward()
        return e.grad

    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g = one()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"value": round(steps / dt, 3), "unit": "gradients/s", "ms_per_gradient": round(dt / steps * 1e3, 2),
            "voxels": int(g.numel()), "orders": "25^3 (M = 12)",
            "per_gradient": "plan build + 3 forward + 3 adjoint solves to 1e-9 + voxel correlation"}


def woodpile(gsm, inputs, steps):
    """Four-layer woodpile (rods of eps 10, 128^3 voxels), Lambda = 0.4
    lambda, M = 31 (63^3 orders, 128^3 FFT grid), 16 seeded directions with a
    transverse drive each in one batched call, complex64 + FP64 refinement to
    1e-9."""
    import torch
    eps = inputs.woodpile(128, 10.0)
    lam, M = 2.5, (31, 31, 31)
    plan = gsm.Plan(eps, (1.0, 1.0, 1.0), M)
    insts = []
    for kh in inputs.random_directions(16, seed=5):
        inst = gsm.make_instance(lam, 2 * np.pi / lam * np.asarray(kh), M, [tuple(inputs.transverse_drive(kh))])
        inst.eps_b = plan.basis_eps(inst)
        insts.append(inst)
    opts = gsm.default_opts(tol=TOL, precision=gsm.GSM_MIXED, restart=30)
    plan.solve(insts, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    worst = 0.0
    for _ in range(steps):
        _, info, st = plan.solve(insts, opts)
        if st != gsm.GSM_OK:
            raise RuntimeError(f"woodpile solve status {st}")
        worst = max(worst, max(i["rel_residual"] for i in info))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gsm.profile_begin()
    plan.solve(insts, opts)
    prof = gsm.profile_end()
    return {"value": round(16 * steps / dt, 3), "unit": "solves/s", "solves_per_step": 16,
            "ms_per_step": round(dt / steps * 1e3, 1), "max_rel_residual": worst,
            "roofline": matvec_hbm(prof), "roofline_fp64_residual": matvec_hbm(prof, "c128"),
            "kernels": kernel_table(prof)}


# Table 1 of the paper: GPU seconds per solve at 16^3 ... 256^3 harmonics
# (FP64, 1e-8, its own GPU of 2013, the largest with host swapping); context
# only, the nearest odd sizes here
TABLE1_PAPER_GPU_S = {7: ("16^3", 0.166), 15: ("32^3", 0.244), 31: ("64^3", 0.448),
                      63: ("128^3", 2.184), 127: ("256^3", 113.676)}


def table1(gsm, inputs, reps):
    """Table 1's workload, one solve per call as in the table: spheres of
    refractive index 3 in air (r = 0.3 Lambda, Lambda = 0.3 lambda), x drive at
    normal incidence, GMRES(30) to a 1e-8 FP64 relative residual, in FP64 and
    in complex64 + FP64 refinement, at 15^3, 31^3, 63^3, 127^3 and 255^3
    harmonics (FFT grids 32 ... 512).  Wall time per call averaged over `reps`
    calls (the table averages ten; three at 255^3), the plan built
    beforehand."""
    import torch
    rows = []
    for M, (orders, paper_s) in TABLE1_PAPER_GPU_S.items():
        w = inputs.sphere_lattice_table1(M)
        lam = w["wavelength"]
        k = 2 * np.pi / lam * np.asarray(w["k_hat"], dtype=np.float64)
        plan = gsm.Plan(w["eps"], w["period"], w["M"])
        inst = gsm.make_instance(lam, k, w["M"], w["drives"])
        inst.eps_b = plan.basis_eps(inst)
        row = {"harmonics": f"{2 * M + 1}^3", "M": M, "P": gsm.fft_size(w["M"]), "eps_b": inst.eps_b,
               "paper_orders": orders, "paper_gpu_ms": paper_s * 1e3}
        n_rep = reps if M < 127 else min(reps, 3)
        row["reps"] = n_rep
        for name, prec in (("fp64", gsm.GSM_FP64), ("mixed", gsm.GSM_MIXED)):
            opts = gsm.default_opts(tol=1e-8, precision=prec, restart=30)
            plan.solve([inst], opts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n_rep):
                _, info, st = plan.solve([inst], opts)
                if st != gsm.GSM_OK:
                    raise RuntimeError(f"Table 1 workload M={M} {name}: status {st}")
            torch.cuda.synchronize()
            row[f"{name}_ms"] = round((time.perf_counter() - t0) / n_rep * 1e3, 3)
            row[f"{name}_iterations"] = info[0]["iterations"]
            row[f"{name}_rel_residual"] = info[0]["rel_residual"]
        rows.append(row)
        plan.close()
    return {"unit": "ms per solve", "tol": 1e-8, "reps": reps, "rows": rows,
            "note": "paper_gpu_ms: the paper's Table 1 (FP64, its 2013 GPU, 16 ... 256 harmonics per axis; the "
                    "256^3 time includes swapping Krylov vectors to host memory), context"}


# Fig. 2 of the paper: cubic air cavities of side Lambda/2 in n = 1.5 and 3.0,
# Lambda = 0.3 lambda; its printed (converged) effective indices, context
FIG2_PAPER_NEFF = {2.25: 1.441688, 9.0: 2.82503}


def pole_search(gsm, steps):
    """The pole search of Eqs.(6)-(10) on Fig. 2's lattices at 31^3
    harmonics (64^3 grid): per host permittivity, the E system (x drive,
    xi = E_x,0) and the H system (y drive, xi = H_y,0) along z, N_p = 5,
    N_d = 10 (15 mesh solves per query, complex64 + FP64 refinement to
    1e-10), all four queries' 60 solves in two calls (one per system); wall
    time per search and the effective indices beside the paper's."""
    import torch
    M = (15, 15, 15)
    lam = 1 / 0.3
    k0 = 2 * np.pi / lam
    out = {"unit": "searches/s", "n_poles": 5, "n_div": 10, "harmonics": "31^3", "rows": []}
    plans, queries = [], []
    for eh, n_paper in FIG2_PAPER_NEFF.items():
        vox = np.full((4, 4, 4), eh)
        vox[1:3, 1:3, 1:3] = 1.0
        plans.append(gsm.Plan(vox, (1.0, 1.0, 1.0), M))
        lo, hi = (n_paper - 0.08) * k0, (n_paper + 0.08) * k0
        queries.append((gsm.make_pole_query(lam, (0, 0, 1), M, lo, hi),
                        gsm.make_pole_query(lam, (0, 0, 1), M, lo, hi, drive=(0, 1, 0), component=1)))
    opts = {"E": gsm.default_opts(tol=1e-10), "H": gsm.default_opts(tol=1e-10, formulation=gsm.GSM_FORM_H)}
    res = {}
    for plan, (qe, qh) in zip(plans, queries):   # warm-up (grids, codelet tuning)
        plan.pole_search([qe], opts["E"])
        plan.pole_search([qh], opts["H"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for i, (plan, (qe, qh)) in enumerate(zip(plans, queries)):
            res[(i, "E")] = plan.pole_search([qe], opts["E"])[0][0]
            res[(i, "H")] = plan.pole_search([qh], opts["H"])[0][0]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for i, (eh, n_paper) in enumerate(FIG2_PAPER_NEFF.items()):
        row = {"host_eps": eh, "paper_n_eff": n_paper}
        for f in ("E", "H"):
            r = res[(i, f)]
            row[f"{f}_n_eff"] = r["n_eff"]
            row[f"{f}_status"] = r["status"]
            row[f"{f}_mesh_iterations"] = r["iterations"]
            row[f"{f}_max_rel_residual"] = r["max_rel_residual"]
        out["rows"].append(row)
    n = 4 * steps
    out["value"] = round(n / dt, 3)
    out["ms_per_search"] = round(dt / n * 1e3, 3)
    for p in plans:
        p.close()
    return out


# Fig. 4 of the paper: spherical air cavities in an n = 1.5 host on a
# tetragonal lattice (Lambda_y = Lambda_z), filling factor 0.155 held fixed
# while Lambda_x / Lambda_yz varies; its Maxwell-Garnett index, context
FIG4_MG_INDEX = 1.4213


def fresnel_tensor(gsm, steps):
    """The paper's tensor retrieval on Fig. 4's uniaxial lattices: cavity
    radius 0.03 lambda, f = 0.155, Lambda_x / Lambda_yz = 0.7 and 1.3
    (analytic sphere images, 15^3 harmonics): the six axis pole searches
    (N_p = 5, N_d = 10, complex64 + FP64 refinement to 1e-10) and the
    diagonal Fresnel fit per lattice; wall time per tensor, the principal
    indices (n_x extraordinary, n_y = n_z ordinary) and the fit's rms."""
    import torch
    M = (7, 7, 7)
    lam, R, f = 1.0, 0.03, 0.155
    out = {"unit": "tensors/s", "harmonics": "15^3", "cavity_radius_over_lambda": R, "fill": f,
           "maxwell_garnett_index": FIG4_MG_INDEX, "rows": []}
    plans = []
    for rho in (0.7, 1.3):
        lyz = (4.0 / 3.0 * np.pi * R ** 3 / (f * rho)) ** (1.0 / 3.0)
        period = (rho * lyz, lyz, lyz)
        sphere = {"kind": "sphere", "centre": tuple(0.5 * p for p in period), "size": R, "eps": 1.0}
        plans.append((rho, period, gsm.Plan.from_shapes(period, 2.25, [sphere], M)))
    opts = gsm.default_opts(tol=1e-10)
    for _, _, plan in plans:                      # warm-up (grids, codelet tuning)
        plan.fresnel_tensor(lam, M, 1.30, 1.55, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = {}
    for _ in range(steps):
        for rho, _, plan in plans:
            res[rho] = plan.fresnel_tensor(lam, M, 1.30, 1.55, opts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for rho, period, plan in plans:
        eps, rms, pairs, _ = res[rho]
        n = np.sqrt(np.diag(eps))
        out["rows"].append({"lambda_x_over_lambda_yz": rho, "period_over_lambda": [round(p, 5) for p in period],
                            "n_x": float(n[0]), "n_y": float(n[1]), "n_z": float(n[2]), "fit_rms": rms,
                            "axis_index_pairs": pairs.tolist()})
        plan.close()
    n_t = len(plans) * steps
    out["value"] = round(n_t / dt, 3)
    out["ms_per_tensor"] = round(dt / n_t * 1e3, 3)
    return out


def hfield_solve(work, gsm, steps):
    """The headline batch (both bodies, 128 solves) through the H-field
    system of Eq.(5) (transverse H drives: the E drives rotated by k x),
    complex64 + FP64 refinement to 1e-9: solves/s beside the E system's."""
    import torch
    opts = gsm.default_opts(tol=TOL, precision=gsm.GSM_MIXED, restart=30, formulation=gsm.GSM_FORM_H)
    hw = []
    for plan, insts in work:
        hi = []
        for inst in insts:
            k = np.array([inst.k_inc[a] for a in range(3)])
            kh = k / np.linalg.norm(k)
            drives = []
            for d in range(inst.n_drive):
                a = np.array([complex(inst.pol[d][2 * c], inst.pol[d][2 * c + 1]) for c in range(3)])
                drives.append(tuple(np.cross(kh, a)))
            h = gsm.make_instance(inst.wavelength, k, [inst.M[a] for a in range(3)], drives)
            h.eps_b = plan.basis_eps(h)
            hi.append(h)
        hw.append((plan, hi))
    for plan, hi in hw:
        plan.solve(hi, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n, worst, iters = 0, 0.0, 0
    for _ in range(steps):
        for plan, hi in hw:
            _, info, st = plan.solve(hi, opts)
            if st != gsm.GSM_OK:
                raise RuntimeError(f"H-field solve status {st}")
            n += len(info)
            worst = max(worst, max(i["rel_residual"] for i in info))
            iters += sum(i["iterations"] for i in info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"value": round(n / dt, 3), "unit": "solves/s", "solves_per_step": n // steps,
            "max_rel_residual": worst, "mean_iterations": round(iters / n, 2)}


def matvec_hbm(prof, prec="c64"):
    """The matrix-vector product as a whole (passes A, B and C of a profiled
    step): algorithmic bytes over the summed launch durations, against the
    HBM peak; the bytes both on the grids in use and on the smallest
    admissible grids (P_min >= 4M + 1, no prime factor above 5: the bytes
    model's, so that a grid larger than needed does not count as work)."""
    parts = [prof.get(f"pass_{x}_{prec}") for x in "abc"]
    if not all(parts):
        return None
    ms = sum(v["ms"] for v in parts)
    gbs = sum(v["bytes"] for v in parts) / (ms * 1e-3) / 1e9
    gbs_min = sum(v["bytes_min"] for v in parts) / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs_min, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs_min / HBM_PEAK_GBS, 4), "bytes": "B_mv on P_min",
            "achieved_grid_in_use": round(gbs, 1), "frac_grid_in_use": round(gbs / HBM_PEAK_GBS, 4),
            "launches": parts[0]["launches"], "ms": round(ms, 3), "precision": prec,
            "per_pass_GBps": {f"pass_{x}": round(v["bytes_min"] / (v["ms"] * 1e-3) / 1e9, 1)
                              for x, v in zip("abc", parts)}}


def host_cpu():
    """CPU model and thread count of the host (for the CPU baseline)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def copy_bandwidth():
    """Achievable HBM rate of a plain shader copy: torch's elementwise negation
    of 2^28 float32 values (read 1 GiB, write 1 GiB), best of five."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.neg(src, out=dst)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    gbs = 2 * (1 << 30) / (best * 1e-3) / 1e9
    return {"GBps": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes": 2 * (1 << 30),
            "kernel": "torch.neg, 1 GiB in + 1 GiB out, best of 5"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(instances shard across GPUs with no communication, see DESIGN.md)"}))
        sys.exit(2)
    import torch

    from paper_1501_01752_amd import gsm, inputs
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device"}))
        sys.exit(1)
    work = build_workload(gsm, inputs, args.directions, autotune=not args.no_autotune)
    bodies = Bodies(work, serial=not args.concurrent_bodies)
    if args.matvec_only:
        matvec_only(gsm, work[0], args.matvec_only, args.matvec_systems)
        return
    extra = {} if args.inner_tol is None else {"inner_tol": args.inner_tol}
    if args.group_max is not None:
        extra["group_max"] = args.group_max
    opts = gsm.default_opts(tol=TOL, precision=gsm.GSM_MIXED, restart=30, **extra)
    for _ in range(args.warmup):
        run_step(gsm, bodies, opts)
    torch.cuda.synchronize()

    # one extra step with every kernel class timed: the per-class table and
    # the dominant class
    gsm.profile_begin()
    run_step(gsm, bodies, opts)
    prof_all = gsm.profile_end()
    kernels = kernel_table(prof_all)
    matvec = matvec_hbm(prof_all)
    step_bytes = sum(v["bytes"] for v in prof_all.values())
    dom_name = next(iter(kernels))
    dom_class = dom_name.rsplit("_", 1)[0]

    for k in STATS:
        STATS[k] = 0
    gsm.profile_begin(only=dom_class if args.profile == "dominant" else None, every=args.profile_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total = 0
    worst = 0.0
    for _ in range(args.steps):
        n, w = run_step(gsm, bodies, opts)
        total += n
        worst = max(worst, w)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = gsm.profile_end()
    krylov = {k: round(STATS[k] / max(1, STATS["solves"]), 2) for k in ("iterations", "refinements", "reorth")}
    dt = t1 - t0
    value = total / dt
    # the whole solve against HBM: the algorithmic bytes of every launch of
    # one step (passes, Gram-Schmidt, least squares, FP64 residuals, each by
    # its definition) over the timed steps' wall time per step
    step_gbs = step_bytes / (dt / args.steps) / 1e9
    step_hbm = {"bound": "hbm", "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(step_gbs / HBM_PEAK_GBS, 4), "bytes_per_step": int(step_bytes),
                "bytes": "algorithmic bytes of every launch of one step, counted on an extra step with every "
                         "launch timed, over the wall time of a timed step"}
    # roofline of the dominant class from its launches in the timed steps
    roofline = roofline_of(dom_name, prof[dom_name])
    roofline["group_max"] = opts.group_max
    rec = counted_traffic(dom_name)

    def add_traffic(r, record):
        r["traffic"] = record["traffic_bytes_per_dispatch"]
        r["traffic_algorithmic"] = record["algorithmic_bytes_per_dispatch"]
        r["traffic_launch"] = record["launch"]

    # counters taken on a launch of as many systems as the timed launches carry
    per_launch = min(opts.group_max or 10 ** 9, len(gsm.system_sizes(work[0][1])))
    rec_launch = counted_traffic(dom_name, per_launch)
    if rec_launch is not None:
        add_traffic(roofline, rec_launch)
    if opts.group_max != 0:
        roofline["note"] = ("the systems of a call run as concurrent launch groups of at most group_max: a "
                            "launch's event duration includes the other groups' concurrent work, so this rate "
                            "is a lower bound of the kernel's own; roofline_one_group times it alone")

    # the same steps with one launch group per call (no concurrent groups):
    # the dominant kernel's own launch rate, and the throughput without
    # splitting, timed on their own
    one_group = None
    og_steps = args.steps if args.one_group_steps is None else args.one_group_steps
    if og_steps > 0 and opts.group_max != 0:
        opts1 = gsm.default_opts(tol=TOL, precision=gsm.GSM_MIXED, restart=30,
                                 **{k: v for k, v in extra.items() if k != "group_max"}, group_max=0)
        run_step(gsm, bodies, opts1)
        gsm.profile_begin(only=dom_class, every=args.profile_every)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        n1 = 0
        for _ in range(og_steps):
            n, _ = run_step(gsm, bodies, opts1)
            n1 += n
        torch.cuda.synchronize()
        t6 = time.perf_counter()
        prof1 = gsm.profile_end()
        one_group = roofline_of(dom_name, prof1[dom_name])
        one_group["group_max"] = 0
        one_group["solves_per_s"] = round(n1 / (t6 - t5), 3)
        one_group["steps"] = og_steps
        if rec is not None:
            add_traffic(one_group, rec)

    # plain FP64 GPU solve of the same workload
    fp64 = None
    if args.fp64_steps > 0:
        opts64 = gsm.default_opts(tol=TOL, precision=gsm.GSM_FP64, restart=30)
        run_step(gsm, bodies, opts64)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        n64 = 0
        for _ in range(args.fp64_steps):
            n, _ = run_step(gsm, bodies, opts64)
            n64 += n
        torch.cuda.synchronize()
        fp64 = {"value": round(n64 / (time.perf_counter() - t2), 3), "unit": "solves/s"}

    # the literal 4-solve case: x, y drives at normal incidence, both bodies
    as_configured = None
    if args.config_steps > 0:
        # latency bound: its two bodies always run concurrently (no roofline is taken here)
        small = Bodies(build_workload(gsm, inputs, 0, autotune=not args.no_autotune), serial=False)
        run_step(gsm, small, opts)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        ns = 0
        for _ in range(args.config_steps):
            n, _ = run_step(gsm, small, opts)
            ns += n
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        as_configured = {"value": round(ns / (t4 - t3), 3), "unit": "solves/s",
                         "bodies": "concurrent (one host thread and stream each)",
                         "solves_per_step": ns // args.config_steps,
                         "ms_per_step": round((t4 - t3) / args.config_steps * 1e3, 3)}

    sweep = uneven_sweep(gsm, inputs, args.sweep_steps, not args.no_autotune) if args.sweep_steps > 0 else None
    design = inverse_design(gsm, inputs, args.design_steps) if args.design_steps > 0 else None
    wood = woodpile(gsm, inputs, args.woodpile_steps) if args.woodpile_steps > 0 else None
    tab1 = table1(gsm, inputs, args.table1_reps) if args.table1_reps > 0 else None
    poles = pole_search(gsm, args.pole_steps) if args.pole_steps > 0 else None
    hfield = hfield_solve(work, gsm, args.hfield_steps) if args.hfield_steps > 0 else None
    fresnel = fresnel_tensor(gsm, args.fresnel_steps) if args.fresnel_steps > 0 else None
    cpu = None if args.no_cpu else cpu_baseline(inputs)
    copy_bw = copy_bandwidth()
    per_step = total // args.steps
    line = {
        "metric": "GSM solves/sec to 1e-9 rel. residual at 31^3 orders; matvec HBM GB/s vs peak",
        "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64",
        "data": "synthetic", "profile": f"{args.profile}, 1 launch in {args.profile_every} timed",
        "config": {"workload": "31^3 orders (M=15), 64^3 FFT grid: sphere lattice (r=0.3 Lambda, eps 4, "
                               "64^3 voxels) + layered stack (f=0.4, eps 2.25/9), Lambda=0.3 lambda, "
                               f"2 transverse drives x (normal incidence + {args.directions} seeded directions) "
                               "per body, batched; complex64 GMRES(30) + FP64 refinement to 1e-9",
                   "solves_per_step": per_step, "max_rel_residual": worst,
                   "codelet_families": {name: work[i][0].tuning(work[i][1][0].M)[0]
                                        for i, name in enumerate(("sphere", "stack"))},
                   "bodies": "concurrent (one host thread and stream each)" if args.concurrent_bodies else "serial",
                   "group_max": opts.group_max,
                   "per_solve_mean": krylov},
        "roofline": roofline,
        "roofline_one_group": one_group,
        "matvec_hbm": matvec,
        "step_hbm": step_hbm,
        "copy_bandwidth": copy_bw,
        "fp64_gpu_solve": fp64,
        "as_configured": as_configured,
        "uneven_sweep": sweep,
        "inverse_design": design,
        "woodpile": wood,
        "table1": tab1,
        "pole_search": poles,
        "hfield_solve": hfield,
        "fresnel_tensor": fresnel,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
