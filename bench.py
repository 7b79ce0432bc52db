"""Benchmark: one semi-smooth Newton step of the phase-field fracture problem.

Workload (default): 2D unit square, 256x256 cells, Q2 for (u_x, u_y, phi)
= 789,507 dofs, FP64; residual, active set, linearisation (diagonals,
Lanczos estimates, coarse factorisation), FGMRES(30) preconditioned by a
5-level monolithic GMG V-cycle to a 1e-8 relative residual, and the update.
Each timed step restarts from the same seeded synthetic state, with all
inputs resident in HBM before timing starts.

Prints one JSON line with the metric, the Newton-step throughput (DoF/s),
the live roofline of the dominant kernel (the finest-level cell kernel,
timed with HIP events on the library's stream) and the oracle timed on the
host cores on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Jacobian-apply DoFs/s and GMG-GMRES time per Newton step, FP64 vs mixed"
HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "rowcell_apply_c2_f64_counters.txt")
N_ROTATE = 8   # contexts the HBM-resident product timing rotates through
KERNEL_SRC = os.path.join(ROOT, "paper_2005_00331_amd", "csrc", "rowcell_kernel.hip")


def measured_traffic(cfg):
    """HBM bytes per launch of the finest-level product, from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (scaled by a 64 MiB copy); None for another workload
    or when the kernel source has changed since the counters were taken."""
    if cfg.name != "C2" or not os.path.exists(COUNTERS):
        return None
    kv = {}
    with open(COUNTERS) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split(None, 1)
                kv[k] = v.strip()
    with open(KERNEL_SRC, "rb") as f:
        src_hash = hashlib.sha256(f.read()).hexdigest()
    if kv.get("kernel_source_sha256") != src_hash:
        return None
    return float(kv["apply_traffic_bytes"])


def algorithmic_bytes_per_apply(dim, n_nodes, elem):
    """x read + y written ((dim+1) comps each), u (dim comps), phi, phi~ read, 1-byte mask."""
    return ((dim + 1) * 2 + dim + 2) * elem * n_nodes + n_nodes


def build_context(cfg, prec=None):
    import torch
    from paper_2005_00331_amd import Context, problem_from
    from synth import level_list, make_inputs
    levels = level_list(cfg)
    ctx = Context(problem_from(cfg, levels, vcycle_prec=prec))
    inp = make_inputs(cfg)

    def d(a):
        return torch.from_numpy(a.ravel().copy()).cuda()
    state = {k: d(v) for k, v in inp.items()}
    return ctx, levels, state


def time_newton(ctx, state, steps, warmup):
    import torch
    u = state["u"].clone()
    phi = state["phi"].clone()
    act = torch.empty_like(state["active"])
    infos = []

    def step():
        u.copy_(state["u"])
        phi.copy_(state["phi"])
        _, info = ctx.newton_step(u, phi, state["phi_old"], state["phi_tilde"], act)
        infos.append(info)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    infos.clear()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps, infos


def time_apply(ctx, n_launch=50, f32=False):
    """Average duration of one finest-level product (full operator, FP64 unless f32), timed
    with HIP events on the stream the library launches on. 2D: one owner-computes kernel;
    3D: the line kernel (element results) plus the node gather."""
    import torch
    from paper_2005_00331_amd import F32, F64, OP_G
    n = ctx.n_dofs
    op = OP_G
    prec, dt = (F32, torch.float32) if f32 else (F64, torch.float64)
    x = torch.randn(n, dtype=dt, device="cuda")
    y = torch.zeros(n, dtype=dt, device="cuda")
    for _ in range(5):
        ctx.apply_jacobian(-1, x, y, prec=prec, op=op)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(n_launch):
        ctx.apply_jacobian(-1, x, y, prec=prec, op=op)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / n_launch


def time_apply_cold(ctx, reps=10):
    """Median duration of one finest-level FP64 product with the 256 MB last-level cache (MALL)
    flushed before each: a 1 GiB buffer is written between the products, and HIP events bracket
    only the product."""
    import torch
    from paper_2005_00331_amd import F64, OP_G
    n = ctx.n_dofs
    x = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    ctx.apply_jacobian(-1, x, y, prec=F64, op=OP_G)
    s = torch.cuda.current_stream()
    times = []
    for rep in range(reps):
        flush.fill_(rep & 0xFF)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        ctx.apply_jacobian(-1, x, y, prec=F64, op=OP_G)
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    del flush
    return sorted(times)[len(times) // 2]


def time_copy_rotating(nbytes, n_pairs=N_ROTATE, rounds=10):
    """Average duration of a plain device copy that moves nbytes of HBM traffic (nbytes / 2 read,
    nbytes / 2 written), rotating through n_pairs buffer pairs like the product: the practical
    floor of a kernel with that many bytes, launch and ramp included."""
    import torch
    n = max(1, int(nbytes // 16))
    pairs = [(torch.ones(n, dtype=torch.float64, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"))
             for _ in range(n_pairs)]
    for a, b in pairs:
        b.copy_(a)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(rounds):
        for a, b in pairs:
            b.copy_(a)
    e1.record(s)
    e1.synchronize()
    del pairs
    return e0.elapsed_time(e1) / 1e3 / (rounds * n_pairs)


def product_contexts(cfg, n_ctx):
    """n_ctx single-level contexts of the workload's finest level at its seeded point (no active
    set), each with its own trial and result vector: together several times the 256 MB
    last-level cache, so that rotating through them makes every product read its operands from
    HBM."""
    import torch
    from paper_2005_00331_amd import Context, problem_from
    from synth import make_inputs
    inp = make_inputs(cfg)

    def d(a):
        return torch.from_numpy(a.ravel().copy()).cuda()
    st = {k: d(v) for k, v in inp.items()}
    out = []
    for _ in range(n_ctx):
        ctx = Context(problem_from(cfg, [(cfg.N, cfg.k)]))
        zeros = torch.zeros(ctx.n_nodes, dtype=torch.uint8, device="cuda")
        ctx.set_point(st["u"], st["phi"], st["phi_old"], zeros, st["phi_tilde"])
        x = torch.randn(ctx.n_dofs, dtype=torch.float64, device="cuda")
        out.append((ctx, x, torch.zeros_like(x)))
    return out


def time_apply_rotating(ctxs, rounds=10):
    """Average duration of one finest-level FP64 product over rounds x len(ctxs) back-to-back
    launches that rotate through independent contexts (HIP events on the library's stream, around
    the whole sequence): each launch finds its operands evicted from the last-level cache by the
    others, so this is the HBM-resident figure without per-launch event overhead."""
    import torch
    from paper_2005_00331_amd import F64, OP_G
    for ctx, x, y in ctxs:
        ctx.apply_jacobian(-1, x, y, prec=F64, op=OP_G)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(rounds):
        for ctx, x, y in ctxs:
            ctx.apply_jacobian(-1, x, y, prec=F64, op=OP_G)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / (rounds * len(ctxs))


def host_cpu():
    """Host processor model (from /proc/cpuinfo) and os.cpu_count()."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def bytes_per_iteration(dim, k, cheb_degree, restart, vcycle_bytes_scale=1.0):
    """Algorithmic HBM bytes per dof of one FGMRES(m) iteration, the lower bound a solve is held
    to: one product (x, y, u, phi, phi~, mask), a V-cycle of 2 s smoothing products plus about
    32 B/dof of Chebyshev vector traffic per product on every level (level sizes summed
    geometrically: 4/3 in 2D, 8/7 in 3D), about 20 B/dof of transfers, and CGS2 over on average
    m/2 basis vectors (two passes reading the basis, about 32 B/dof per vector).
    vcycle_bytes_scale = 0.5 for an FP32 V-cycle."""
    apply_b = ((dim + 1) * 2 + dim + 2) * 8 / (dim + 1)
    lsum = 4 / 3 if dim == 2 else 8 / 7
    vc = (2 * cheb_degree * (apply_b + 32) * lsum + 20) * vcycle_bytes_scale
    return apply_b + vc + 32 * restart / 2


def time_autograd(cfg, reps=5, warmup=2):
    """The residual as a torch.autograd.Function (forward R(u, phi; Gc, eps), hand-written backward:
    the point's coefficient cache, the transposed product and the two parameter cotangents) on the
    workload's seeded state and cotangent; medians of wall times with the device synchronised
    around each part, and the ratio of forward + backward to one finest-level product."""
    import torch
    from paper_2005_00331_amd import Context, problem_from
    from paper_2005_00331_amd.autograd import residual
    from synth import make_inputs
    ctx = Context(problem_from(cfg, [(cfg.N, cfg.k)]))
    inp = make_inputs(cfg, ("cotangent",))

    def d(a):
        return torch.from_numpy(a.ravel().copy()).cuda()
    u0, phi0, pt, v = d(inp["u"]), d(inp["phi"]), d(inp["phi_tilde"]), d(inp["cotangent"])
    Gc = torch.tensor(cfg.Gc, dtype=torch.float64, requires_grad=True)
    eps = torch.tensor(cfg.eps, dtype=torch.float64, requires_grad=True)
    fwd, bwd = [], []
    for rep in range(warmup + reps):
        u = u0.clone().requires_grad_(True)
        phi = phi0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R = residual(u, phi, Gc, eps, pt, ctx)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        R.backward(v)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rep >= warmup:
            fwd.append(t1 - t0)
            bwd.append(t2 - t1)
    tf, tb = sorted(fwd)[len(fwd) // 2], sorted(bwd)[len(bwd) // 2]
    t_apply = time_apply(ctx)
    out = {"workload": f"{cfg.name}: 3D {cfg.N}^3 cells Q{cfg.k}, {ctx.n_dofs} dofs, no constraints",
           "ms_forward": tf * 1e3, "ms_backward": tb * 1e3,
           "dofs_per_s_forward_backward": ctx.n_dofs / (tf + tb), "apply_us": t_apply * 1e6,
           "forward_backward_in_products": (tf + tb) / t_apply}
    ctx.close()
    return out


def time_solve(cfg, prec, warm=True):
    """One linear solve of the workload's seeded right-hand side at its seeded state and active
    set: set_linearization, then FGMRES to the workload's rtol (after one untimed warm-up solve
    when warm). FP64 GMRES either way; prec selects the V-cycle precision. The time is set against
    the HBM lower bound iterations x bytes_per_iteration x n_dofs / 8 TB/s."""
    import torch
    from synth import make_inputs
    ctx, levels, state = build_context(cfg, prec=prec)
    rhs = torch.from_numpy(make_inputs(cfg, ("rhs",))["rhs"]).cuda()
    args = (state["u"], state["phi"], state["phi_old"], state["active"], state["phi_tilde"])
    if warm:
        ctx.set_linearization(*args)
        ctx.gmres_solve(rhs, raise_on_noconv=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.set_linearization(*args)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, st = ctx.gmres_solve(rhs, raise_on_noconv=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.close()
    b_it = bytes_per_iteration(cfg.dim, cfg.k, cfg.cheb_degree, cfg.restart, 0.5 if prec == "f32" else 1.0)
    bound_ms = st["iterations"] * b_it * cfg.n_dofs / (HBM_PEAK_GBS * 1e9) * 1e3
    return {"ms_setup": (t1 - t0) * 1e3, "ms_solve": (t2 - t1) * 1e3, "ms_total": (t2 - t0) * 1e3,
            "gmres_iterations": st["iterations"], "converged": st["converged"], "rel_residual": st["rel_residual"],
            "active_fraction": float(state["active"].float().mean()),
            "bytes_per_dof_per_iteration": b_it, "hbm_bound_ms": bound_ms,
            "solve_frac_of_hbm_bound": bound_ms / ((t2 - t1) * 1e3)}


def contraction_flops_3d(cfg):
    """FP64/FP32 flops of the sum-factorised contractions of one 3D product in the line
    kernel: per cell 33 (k+1)^4 multiply-adds forward (x, y, z steps over four fields)
    and 33 (k+1)^4 backward; the point physics (about 100 flops per Gauss point) is not
    counted."""
    n_cells = cfg.N ** 3
    return 2 * 66 * (cfg.k + 1) ** 4 * n_cells


def time_products_3d(cfg):
    """Finest-level product of a 3D workload in FP64 and FP32 after set_linearization."""
    ctx, levels, state = build_context(cfg, prec="f32")
    ctx.set_linearization(state["u"], state["phi"], state["phi_old"], state["active"], state["phi_tilde"])
    engine = "matrix cores (MFMA)" if cfg.contraction == "mfma" and cfg.k >= 3 else "vector unit"
    fl = contraction_flops_3d(cfg)
    res = {"workload": f"{cfg.name}: 3D {cfg.N}^3 cells Q{cfg.k}, {cfg.n_dofs} dofs, finest-level product "
                       f"(cell kernel + node gather)", "contractions_on": engine, "contraction_gflop": fl / 1e9,
           "note": "operands, coefficient cache and element buffer exceed the 256 MB last-level cache, so "
                   "back-to-back launches read from HBM; frac_of_peak counts only the contraction flops"}
    for f32, tag, peak in ((False, "f64", 78.6), (True, "f32", 157.3)):
        t = time_apply(ctx, f32=f32)
        byts = algorithmic_bytes_per_apply(cfg.dim, ctx.n_nodes, 4 if f32 else 8)
        res[tag] = {"apply_us": t * 1e6, "dofs_per_s": ctx.n_dofs / t, "contraction_tflops": fl / t / 1e12,
                    "frac_of_peak": fl / t / 1e12 / peak, "peak_tflops": peak,
                    "algorithmic_bytes": byts, "hbm_GBps": byts / t / 1e9,
                    "hbm_frac": byts / t / 1e9 / HBM_PEAK_GBS}
    ctx.close()
    return res


def spmv_study():
    """Section 6's comparison on this GPU: per degree, the matrix-free product (unconstrained,
    cached coefficients where the level has them; back to back, cache-resident, and rotating
    through contexts, HBM-resident) against the sparse product of the assembled
    Jacobian (CSR with 32-bit indices, rocSPARSE's generic SpMV, the fastest of its adaptive,
    row-split and LRB algorithms), at about the
    same number of dofs; memory per dof of each.  Prints one JSON line per case."""
    import torch
    from paper_2005_00331_amd import OP_G
    from paper_2005_00331_amd.assembly import RocsparseSpmv, assemble_csr
    from synth import CONFIGS
    cases = [(2, 512, 1), (2, 256, 2), (2, 170, 3), (2, 128, 4), (3, 64, 1), (3, 32, 2), (3, 21, 3), (3, 16, 4)]
    for dim, N, k in cases:
        base = CONFIGS["C2"] if dim == 2 else CONFIGS["C3"]
        cfg = base.with_(N=N, k=k, n_h_levels=1, p_coarse=(), dirichlet=False, vcycle_prec="f64")
        ctx, _, st = build_context(cfg)
        zeros = torch.zeros(ctx.n_nodes, dtype=torch.uint8, device="cuda")
        ctx.set_point(st["u"], st["phi"], st["phi_old"], zeros, st["phi_tilde"])
        t_mf = time_apply(ctx)
        # the same product with its operands in HBM (rotating through contexts that together
        # exceed the last-level cache), the regime the CSR matrices (>= 258 MB) are always in
        rot = product_contexts(cfg, N_ROTATE)
        t_mf_hbm = time_apply_rotating(rot)
        for c_, _, _ in rot:
            c_.close()
        del rot
        torch.cuda.empty_cache()
        em = ctx.element_matrices(-1)
        A = assemble_csr(em, dim, N, k)
        del em
        torch.cuda.empty_cache()
        x = torch.randn(ctx.n_dofs, dtype=torch.float64, device="cuda")
        ymf = ctx.apply_jacobian(-1, x, op=OP_G)
        t_sp, alg_best, err = None, None, None
        for alg in ("adaptive", "rowsplit", "lrb"):
            sp = RocsparseSpmv(A, alg)
            sp.x.copy_(x)
            y = sp.mv()
            e = float((y - ymf).norm() / ymf.norm())
            for _ in range(3):
                sp.mv()
            s = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(20):
                sp.mv()
            e1.record(s)
            e1.synchronize()
            t = e0.elapsed_time(e1) / 1e3 / 20
            sp.close()
            del sp
            if t_sp is None or t < t_sp:
                t_sp, alg_best, err = t, alg, e
        nnz = A.values().numel()
        n = ctx.n_dofs
        csr_bytes = nnz * 12 + (n + 1) * 4
        qd = 0
        if (dim == 2 and k <= 2) or dim == 3:
            P = (k + 1) ** dim
            ncoef = 5 if dim == 2 else 8
            qd = N ** dim * P * ncoef * 8 * (64 / 49 if dim == 2 else 1)
        out = {"dim": dim, "N": N, "k": k, "n_dofs": n, "nnz": nnz, "nnz_per_row": nnz / n,
               "mf_us": t_mf * 1e6, "mf_us_hbm": t_mf_hbm * 1e6, "spmv_us": t_sp * 1e6,
               "spmv_over_mf": t_sp / t_mf, "spmv_over_mf_hbm": t_sp / t_mf_hbm,
               "csr_bytes_per_dof": csr_bytes / n, "spmv_GBs": (csr_bytes + 16 * n) / t_sp / 1e9,
               "mf_state_bytes_per_dof": (algorithmic_bytes_per_apply(dim, ctx.n_nodes, 8) - 16 * n) / n,
               "mf_cache_bytes_per_dof": qd / n, "csr_vs_mf_rel_diff": err, "spmv_alg": alg_best}
        print(json.dumps(out), flush=True)
        del A, x, y, ymf
        ctx.close()
        torch.cuda.empty_cache()


def cpu_baseline(cfg_name):
    """Oracle Newton step on a bounded sample of the same workload family."""
    import numpy as np
    from oracle import newton
    from synth import CONFIGS, level_list, make_inputs
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas_threads = os.cpu_count()
    model, ncpu = host_cpu()
    base = CONFIGS[cfg_name]
    cfg = base.with_(N=base.N // 2, n_h_levels=base.n_h_levels - 1)   # same coarse grid, 1/4 of the dofs
    inp = make_inputs(cfg)
    t0 = time.perf_counter()
    out = newton.newton_step(cfg, level_list(cfg), inp["u"], inp["phi"], inp["phi_old"], inp["phi_tilde"])
    t = time.perf_counter() - t0
    return {"value": cfg.n_dofs / t, "unit": "DoF/s", "cores": int(blas_threads), "kind": "oracle",
            "sample": (f"one oracle Newton step (assembly, {cfg.n_h_levels}-level GMG hierarchy, FGMRES) on "
                       f"{cfg.N}x{cfg.N} Q{cfg.k}, {cfg.n_dofs} dofs, {t:.1f} s, {out['info']['iterations']} GMRES "
                       f"iterations; sparse products single-threaded, dense coarse factorisation on "
                       f"{blas_threads} BLAS threads"),
            "seconds": t, "iterations": out["info"]["iterations"], "host_model": model, "host_cpu_count": ncpu,
            "blas_threads": int(blas_threads), "sparse_threads": 1}


def load_steps_detail(ctx, cfg, n_steps=3, du=1e-5):
    """Load steps of the tension test (top face pulled by t du along the last axis) from rest with
    phi = 1 off the notch: first a step with no load, in which the phi = 0 band relaxes into the
    phase-field profile around it (otherwise the extrapolation from the sharp band to the profile
    overshoots), then n_steps loaded steps; per step the loop's counts, time and top reaction."""
    import torch
    from synth.fields import make_phi
    u = torch.zeros(cfg.dim * cfg.n_nodes, dtype=torch.float64, device="cuda")
    p_prev, p_prev2 = torch.tensor(make_phi(cfg.with_(phi_mode="ones")), device="cuda"), None
    direction = [0.0] * (cfg.dim - 1) + [1.0]
    rec = []
    for t in range(0, n_steps + 1):
        phi = p_prev.clone()
        _, info = ctx.load_step(u, phi, p_prev, p_prev2, [t * du * a for a in direction], max_newton=20, tol=1e-8,
                                raise_on_noconv=False)
        rec.append({"u_top": t * du, "newton_steps": info["newton_steps"], "converged": info["converged"],
                    "gmres_iterations": info["gmres_iterations"], "ms": info["ms_total"],
                    "reaction_top": info["reaction_top"][-1]})
        # the relaxation step is not part of the load history
        p_prev2, p_prev = (None, phi) if t == 0 else (p_prev, phi)
    loaded = rec[1:]
    return {"du": du, "relaxation_step": rec[0], "steps": loaded,
            "ms_per_load_step": sum(r["ms"] for r in loaded) / len(loaded)}


def slit_curve(N=64, du=1.5e-4, max_steps=100, coarse_N=None, max_iter=5000, rtol=None):
    """The single-edge-notched tension test of Section 5 on the slit mesh of Section 5.1: 2D Q1,
    N x N cells, the slit along the mid-plane for x < 1/2 as duplicated nodes, phi = 1 at rest,
    the top face pulled by t du (bottom fixed); one level, whose exact coarse solve preconditions
    FGMRES, or with coarse_N the multigrid hierarchy of slit meshes coarse_N, 2 coarse_N, ..., N;
    Algorithm 1 with the projected update in every load step, FGMRES capped at max_iter iterations
    and stopped at rtol (the workload's 1e-8 by default; Section 6 solves to 1e-6).  Runs until the top reaction
    has fallen below 5 % of its peak (the crack has crossed the specimen) or max_steps; per step
    the prescribed displacement, the reaction, Newton steps, FGMRES iterations, active nodes and
    time.  The paper's own curve is a figure without data, so the comparison is qualitative."""
    import torch
    from paper_2005_00331_amd import Context, problem_from
    from synth import CONFIGS
    cfg = CONFIGS["C1"].with_(N=N, n_h_levels=1, p_coarse=(), slit=True, phi_mode="ones", pdas_project=True,
                              max_iter=max_iter)
    if rtol is not None:
        cfg = cfg.with_(rtol=rtol)
    levels = [(N, 1)]
    while coarse_N and levels[0][0] > coarse_N:
        levels.insert(0, (levels[0][0] // 2, 1))
    ctx = Context(problem_from(cfg, levels))
    u = torch.zeros(cfg.dim * cfg.n_nodes, dtype=torch.float64, device="cuda")
    p_prev, p_prev2 = torch.ones(cfg.n_nodes, dtype=torch.float64, device="cuda"), None
    rec, peak = [], 0.0
    t0 = time.perf_counter()
    for t in range(1, max_steps + 1):
        phi = p_prev.clone()
        act, info = ctx.load_step(u, phi, p_prev, p_prev2, [0.0, t * du], max_newton=40, tol=1e-8,
                                  raise_on_noconv=False)
        F = info["reaction_top"][-1]
        rec.append({"u_top": t * du, "reaction_top": F, "newton_steps": info["newton_steps"],
                    "converged": info["converged"], "rel_residual": info["rel_residual"],
                    "gmres_iterations": info["gmres_iterations"],
                    "n_active": int(act.sum().item()), "phi_min": float(phi.min().item()), "ms": info["ms_total"]})
        print(f"[bench] slit load step {t}: u_top {t * du:.4g} reaction {F:.5g} newton {info['newton_steps']} "
              f"active {rec[-1]['n_active']} phi_min {rec[-1]['phi_min']:.3g}", file=sys.stderr, flush=True)
        p_prev2, p_prev = p_prev, phi
        peak = max(peak, F)
        if t > 5 and F < 0.05 * peak:
            break
        if not info["converged"] and not info["rel_residual"] <= 1e-6:
            break  # far from an equilibrium (the linear solves failed): the curve ends here
    ctx.close()
    ip = max(range(len(rec)), key=lambda i: rec[i]["reaction_top"])
    return {"workload": f"single-edge-notched tension, slit mesh: 2D {N}^2 cells Q1, {cfg.n_dofs} dofs "
                        f"({cfg.n_nodes - (N + 1) ** 2} duplicated slit nodes), eps = {cfg.eps:g}, du = {du:g}, "
                        f"levels N = {[n for n, _ in levels]}, FGMRES rtol {cfg.rtol:g}",
            "peak_reaction": rec[ip]["reaction_top"], "u_top_at_peak": rec[ip]["u_top"],
            "all_converged": all(r["converged"] for r in rec),
            "steps": rec, "seconds": time.perf_counter() - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison step")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D runs (C3 solves, C4 products)")
    ap.add_argument("--spmv", action="store_true",
                    help="instead: matrix-free product against the assembled CSR product (rocSPARSE) at p = 1..4")
    ap.add_argument("--load-steps", action="store_true",
                    help="instead: the C2 load steps (relaxation step, then three loaded steps) with both "
                         "active-set updates, printed as one record")
    ap.add_argument("--slit-curve", action="store_true",
                    help="instead: the load-displacement curve of the notched tension test on the slit mesh")
    ap.add_argument("--slit-N", type=int, default=64, help="with --slit-curve: cells per direction")
    ap.add_argument("--slit-coarse", type=int, default=None,
                    help="with --slit-curve: coarsest multigrid level's cells per direction (default: one level)")
    ap.add_argument("--slit-rtol", type=float, default=None,
                    help="with --slit-curve: FGMRES relative tolerance (default: the workload's)")
    ap.add_argument("--autograd", action="store_true",
                    help="instead: time the C5 residual forward and backward (autograd) and print that record")
    ap.add_argument("--solve", metavar="WORKLOAD",
                    help="instead: one linear solve (set-up plus FGMRES) of the named workload's seeded system with "
                         "the FP64 and the FP32 V-cycle, printed as one record")
    ap.add_argument("--restart", type=int, default=None, help="with --solve: FGMRES restart length (default: the workload's)")
    ap.add_argument("--cheb-degree", type=int, default=None, help="with --solve: Chebyshev degree (default: the workload's)")
    ap.add_argument("--max-iter", type=int, default=5000, help="with --solve: FGMRES iteration cap")
    ap.add_argument("--phi", default=None, choices=("ones", "smooth"),
                    help="with --solve: the phase field off the notch (default: the workload's)")
    ap.add_argument("--contraction", default=None, choices=("valu", "mfma"),
                    help="with --solve or --apply-only: 3D Q3/Q4 contractions on the vector unit or the matrix cores")
    ap.add_argument("--apply-only", action="store_true",
                    help="only time the finest-level cell kernel (for kernel-trace and counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(sharding over several GPUs is a design only)", file=sys.stderr)
        sys.exit(2)
    import torch
    from synth import CONFIGS, level_list
    torch.cuda.set_device(0)
    if args.spmv:
        spmv_study()
        return
    if args.autograd:
        print(json.dumps(time_autograd(CONFIGS["C5"])), flush=True)
        return
    if args.slit_curve:
        print(json.dumps(slit_curve(N=args.slit_N, coarse_N=args.slit_coarse, rtol=args.slit_rtol)), flush=True)
        return
    if args.solve:
        cfg = CONFIGS[args.solve].with_(max_iter=args.max_iter)
        for key, val in (("restart", args.restart), ("cheb_degree", args.cheb_degree), ("contraction", args.contraction),
                         ("phi_mode", args.phi)):
            if val is not None:
                cfg = cfg.with_(**{key: val})
        rec = {"workload": f"{cfg.name}: {cfg.dim}D {cfg.N}^{cfg.dim} cells Q{cfg.k}, {cfg.n_dofs} dofs, levels "
                           f"{level_list(cfg)}, seeded state, active set and right-hand side, rtol {cfg.rtol}",
               "restart": cfg.restart, "cheb_degree": cfg.cheb_degree, "contraction": cfg.contraction,
               "phi_mode": cfg.phi_mode}
        for prec in ("f64", "f32"):
            rec[prec + "_vcycle"] = time_solve(cfg, prec, warm=False)
            print(f"[bench] {cfg.name} solve, {prec} V-cycle: {rec[prec + '_vcycle']}", file=sys.stderr, flush=True)
        print(json.dumps(rec), flush=True)
        return
    if args.load_steps:
        from paper_2005_00331_amd import Context, problem_from
        from synth import level_list
        cfg = CONFIGS["C2"]
        rec = {}
        for name, project in (("as_written", False), ("projected", True)):
            ctx = Context(problem_from(cfg.with_(pdas_project=project), level_list(cfg)))
            rec[name] = load_steps_detail(ctx, cfg)
            ctx.close()
        print(json.dumps(rec), flush=True)
        return
    cfg = CONFIGS[args.workload]
    print(f"[bench] workload {cfg.name}: {cfg.dim}D N={cfg.N} Q{cfg.k}, {cfg.n_dofs} dofs", file=sys.stderr, flush=True)
    ctx, levels, state = build_context(cfg)
    if args.apply_only:
        # calibration for the traffic counters: one plain device copy of 64 MiB
        src = torch.ones(8 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        ctx.close()
        if cfg.dim == 2:
            ctxs = product_contexts(cfg, N_ROTATE)
            t_apply = time_apply_rotating(ctxs)
            byts = algorithmic_bytes_per_apply(cfg.dim, ctxs[0][0].n_nodes, 8)
            print(json.dumps({"apply_us": t_apply * 1e6, "GB/s": byts / t_apply / 1e9, "bytes_per_launch": byts,
                              "timing": f"rotating through {N_ROTATE} contexts"}), flush=True)
            for c, _, _ in ctxs:
                c.close()
        else:
            # 3D: the finest-level product in FP64, then FP32 (50 back-to-back launches each; the
            # operands, coefficient cache and element buffer exceed the last-level cache)
            if args.contraction:
                cfg = cfg.with_(contraction=args.contraction)
            print(json.dumps(time_products_3d(cfg)), flush=True)
        return
    sec, infos = time_newton(ctx, state, args.steps, args.warmup)
    print(f"[bench] newton step {sec * 1e3:.2f} ms, iters {[i['iterations'] for i in infos]}", file=sys.stderr,
          flush=True)
    t_warm = time_apply(ctx)
    elem = 8
    byts = algorithmic_bytes_per_apply(cfg.dim, ctx.n_nodes, elem)
    print(f"[bench] finest cell kernel, cache-resident {t_warm * 1e6:.1f} us", file=sys.stderr, flush=True)
    t_cold = time_apply_cold(ctx)
    print(f"[bench] finest cell kernel after a cache flush {t_cold * 1e6:.1f} us", file=sys.stderr, flush=True)
    ctxs = product_contexts(cfg, N_ROTATE)
    t_apply = time_apply_rotating(ctxs)
    for c, _, _ in ctxs:
        c.close()
    del ctxs
    torch.cuda.empty_cache()
    achieved = byts / t_apply / 1e9
    print(f"[bench] finest cell kernel from HBM (rotating) {t_apply * 1e6:.1f} us, {achieved:.0f} GB/s", file=sys.stderr,
          flush=True)
    t_copy = time_copy_rotating(byts)
    print(f"[bench] plain copy of the same bytes (rotating) {t_copy * 1e6:.1f} us, {byts / t_copy / 1e9:.0f} GB/s",
          file=sys.stderr, flush=True)
    detail = {
        "apply_dofs_per_s": ctx.n_dofs / t_apply,
        "apply_us": t_apply * 1e6,
        "apply_us_cache_resident": t_warm * 1e6,
        "apply_GBps_cache_resident": byts / t_warm / 1e9,
        "apply_us_after_cache_flush": t_cold * 1e6,
        "apply_GBps_after_cache_flush": byts / t_cold / 1e9,
        # the practical floor for a kernel moving the product's algorithmic bytes: a plain copy of
        # as many bytes, also rotating (launch and ramp included)
        "copy_us_same_bytes": t_copy * 1e6,
        "copy_GBps_same_bytes": byts / t_copy / 1e9,
        "apply_frac_of_copy_floor": t_copy / t_apply,
        "gmres_iterations": infos[-1]["iterations"],
        "ms_setup": infos[-1]["ms_setup"],
        "ms_solve": infos[-1]["ms_solve"],
        "rel_residual": infos[-1]["rel_residual"],
        "n_active": infos[-1]["n_active"],
        "active_fraction": infos[-1]["n_active"] / ctx.n_nodes,
    }
    # the linear solve alone at the workload's seeded active set (about 5 % of the phi-dofs), both
    # V-cycle precisions: the Newton step's own active set comes from the rule of Algorithm 1
    for prec in ("f64", "f32"):
        detail[f"linear_solve_seeded_active_{prec}_vcycle"] = time_solve(cfg, prec)
        print(f"[bench] {cfg.name} linear solve at the seeded active set, {prec} V-cycle: "
              f"{detail[f'linear_solve_seeded_active_{prec}_vcycle']}", file=sys.stderr, flush=True)
    if not args.no_mixed:
        mctx, _, mstate = build_context(cfg, prec="f32")
        msec, minfos = time_newton(mctx, mstate, 2, 1)
        detail["mixed_f32_vcycle"] = {"ms_per_step": msec * 1e3, "gmres_iterations": minfos[-1]["iterations"],
                                      "ms_setup": minfos[-1]["ms_setup"], "ms_solve": minfos[-1]["ms_solve"],
                                      "rel_residual": minfos[-1]["rel_residual"]}
        print(f"[bench] mixed newton step {msec * 1e3:.2f} ms", file=sys.stderr, flush=True)
        mctx.close()
    if not args.no_mixed:
        # Algorithm 1 to its stopping test from the same state (one load step)
        import torch
        pu, pphi = state["u"].clone(), state["phi"].clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, pinfo = ctx.pdas_solve(pu, pphi, state["phi_old"], state["phi_tilde"], max_newton=20, tol=1e-8,
                                  raise_on_noconv=False)
        torch.cuda.synchronize()
        pinfo["ms_wall"] = (time.perf_counter() - t0) * 1e3
        detail["active_set_loop"] = pinfo
        print(f"[bench] active-set loop: {pinfo}", file=sys.stderr, flush=True)
        # load stepping (Section 5 loading, Section 3 extrapolation): three steps of the tension
        # test's increment from rest, phi = 1 off the notch, with Algorithm 1's update as written
        # and with the projected update
        from paper_2005_00331_amd import Context, problem_from
        detail["load_steps"] = {"as_written": load_steps_detail(ctx, cfg)}
        pctx = Context(problem_from(cfg.with_(pdas_project=True), levels))
        detail["load_steps"]["projected"] = load_steps_detail(pctx, cfg)
        pctx.close()
        print(f"[bench] load steps: {detail['load_steps']}", file=sys.stderr, flush=True)
        # the same Newton step with the spectral (Miehe) split of Section 2.1
        sctx, _, sstate = build_context(cfg.with_(split="miehe"))
        ssec, sinfos = time_newton(sctx, sstate, 2, 1)
        st_apply = time_apply(sctx)
        detail["miehe_split"] = {"ms_per_step": ssec * 1e3, "gmres_iterations": sinfos[-1]["iterations"],
                                 "ms_setup": sinfos[-1]["ms_setup"], "ms_solve": sinfos[-1]["ms_solve"],
                                 "rel_residual": sinfos[-1]["rel_residual"], "apply_us": st_apply * 1e6,
                                 "apply_dofs_per_s": sctx.n_dofs / st_apply}
        print(f"[bench] miehe-split newton step {ssec * 1e3:.2f} ms, product {st_apply * 1e6:.1f} us", file=sys.stderr,
              flush=True)
        sctx.close()
    if not args.no_3d:
        c3 = CONFIGS["C3"]
        res = {"workload": f"C3: 3D {c3.N}^3 cells Q{c3.k}, {c3.n_dofs} dofs, seeded random right-hand side, "
                           f"seeded 5 % active set, Chebyshev degree {c3.cheb_degree}, {c3.n_h_levels}-level "
                           f"GMG-GMRES({c3.restart}), rtol {c3.rtol}"}
        for prec in ("f64", "f32"):
            res[prec + "_vcycle"] = time_solve(c3, prec)
            print(f"[bench] C3 solve, phi = 1 off the notch, {prec} V-cycle: {res[prec + '_vcycle']}", file=sys.stderr,
                  flush=True)
        # the smooth seeded phi field in [0, 1] off the notch (the input recipe of the C2-C5 workloads)
        c3s = c3.with_(phi_mode="smooth", max_iter=2000)
        for prec in ("f64", "f32"):
            res["smooth_phi_" + prec + "_vcycle"] = time_solve(c3s, prec, warm=False)
            print(f"[bench] C3 solve, smooth phi, {prec} V-cycle: {res['smooth_phi_' + prec + '_vcycle']}",
                  file=sys.stderr, flush=True)
        detail["c3_solve"] = res
        c3p = time_products_3d(c3)
        print(f"[bench] C3 products: {c3p}", file=sys.stderr, flush=True)
        detail["c3_products"] = c3p
        c4 = time_products_3d(CONFIGS["C4"])
        print(f"[bench] C4 products: {c4}", file=sys.stderr, flush=True)
        detail["c4_products"] = c4
        c5 = time_autograd(CONFIGS["C5"])
        print(f"[bench] C5 residual forward/backward: {c5}", file=sys.stderr, flush=True)
        detail["c5_autograd"] = c5
    out = {
        "metric": METRIC,
        "value": ctx.n_dofs / sec,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.dim}D {cfg.N}^{cfg.dim} cells Q{cfg.k}, {cfg.n_dofs} dofs, one "
                               f"semi-smooth Newton step, {len(levels)}-level GMG-GMRES({cfg.restart}), rtol {cfg.rtol}",
                   "levels": levels, "n_dofs": ctx.n_dofs, "vcycle_prec": cfg.vcycle_prec,
                   "active_fraction": detail["active_fraction"],
                   "active_set": "Algorithm 1's rule at the seeded state"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(cfg),
                     "kernel": ((f"rowcell_kernel_2d<{cfg.k},double,APPLY,EPI_APPLY>" if cfg.k <= 2 else
                                 f"tile_kernel_2d<{cfg.k},double,APPLY,EPI_APPLY>") if cfg.dim == 2 else
                                f"linecell_kernel<{cfg.k},double,APPLY> + gather3d_kernel") + " on the finest level",
                     "bytes_per_launch": byts,
                     "timing": f"{N_ROTATE} x 10 back-to-back launches rotating through {N_ROTATE} independent "
                               "contexts (about 53 MB of operands each, together above the 256 MB last-level "
                               "cache), HIP events around the sequence; detail.apply_us_cache_resident is the "
                               "same product repeated on one context"},
        "detail": detail,
    }
    ctx.close()
    if not args.no_cpu:
        print("[bench] oracle cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg.name)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
