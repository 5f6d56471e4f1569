"""Throughput of the DtN-ABC time stepper on one MI355X.

A step is one fourth-order Taylor step of the whole hot path (interior
stencil + potential, boundary operators, auxiliary boundary variables, all
four stages) over the full grid.  Default workload: one orbital on a 128^3
grid, h = 0.2, dt = 0.002, static Gaussian well V = -5 exp(-|x|^2/2), packet
with k = (3, 1, 0) from a seeded centre, first-order face-form condition,
complex128.  Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  Besides throughput it reports the roofline of the
dominant kernel (HIP events over the timed region), the FP64 oracle timed on
the host on a bounded sample, and the physics error of the absorbing run
against a run on a box twice as large per axis with zero boundary values
(same h, dt, integrator; reflections from its walls cannot return in time).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype c128|c64]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def large_box_reference(Solver, torch, wl, path, steps_total):
    """The doubled zero-boundary box run from the zero-extended data, cut back
    to the small box.  Always complex128 with a float64 potential, whatever
    precision the run it is compared with uses."""
    n = wl.n
    big = 2 * n
    off = (big - n) // 2
    from paper_1908_02456_amd import workloads as W
    # zero-extended initial data; the well is evaluated on the big grid
    psi_b = torch.zeros((big, big, big), dtype=torch.complex128, device="cuda")
    psi_b[off:off + n, off:off + n, off:off + n] = torch.from_numpy(wl.psi0)
    Vb = torch.from_numpy(W.gaussian_well((big,) * 3, wl.h, 5.0)).cuda()
    sb = Solver((big,) * 3, wl.h, wl.dt, radius=wl.radius, order="dirichlet", dtype="c128", path=path)
    sb.step(psi_b, None, Vb, steps_total)
    return psi_b[off:off + n, off:off + n, off:off + n].clone()


def physics_error(Solver, torch, wl, dtype, window, path, steps_total, fejer=True):
    """Relative L2 error at T of the absorbing run vs the doubled Dirichlet box
    (complex128), both started from the same box-only data (zero outside the
    small box)."""
    n = wl.n
    big = 2 * n
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    rdt = torch.float64 if dtype == "c128" else torch.float32
    ref = large_box_reference(Solver, torch, wl, path, steps_total)
    s = Solver((n,) * 3, wl.h, wl.dt, radius=wl.radius, order="first", s1=wl.s1, window=window, fejer=fejer,
               dtype=dtype, path=path)
    psi = torch.from_numpy(wl.psi0).to(cdt).cuda()
    aux = s.new_aux()
    V = torch.from_numpy(wl.V).to(rdt).cuda()
    s.step(psi, aux, V, steps_total)
    # the same box with zero boundary values (what the condition replaces)
    sd = Solver((n,) * 3, wl.h, wl.dt, radius=wl.radius, order="dirichlet", dtype=dtype, path=path)
    psid = torch.from_numpy(wl.psi0).to(cdt).cuda()
    sd.step(psid, None, V, steps_total)
    torch.cuda.synchronize()
    nr = torch.linalg.vector_norm(ref).item()
    e_abc = torch.linalg.vector_norm(psi.to(torch.complex128) - ref).item() / nr
    e_dir = torch.linalg.vector_norm(psid.to(torch.complex128) - ref).item() / nr
    h3 = wl.h ** 3
    return {"err_vs_large_box": e_abc, "err_dirichlet_same_box": e_dir, "large_box_n": big,
            "large_box_dtype": "c128", "T": steps_total * wl.dt,
            "norm_abc": h3 * float(torch.sum(torch.abs(psi.to(torch.complex128)) ** 2)),
            "norm_large_box_in_box": h3 * nr * nr, "norm_initial": h3 * float(np.sum(np.abs(wl.psi0) ** 2))}


def shell_counts(n, R):
    """Points within one layer of a face (depth <= 1) and face-slab entries of a cube of side n."""
    inner = max(n - 4, 0) ** 3
    return n ** 3 - inner, 6 * R * n * n


def method_bytes_per_update(n, R, csz, rsz, first=True):
    """Algorithmic bytes of one grid-point update (one point advanced one full
    step, all four stages and the condition): the state read and written once
    (2 csz), the potential read once (rsz) and, for the first order, the FP64
    face aux read and written once (32 B per face entry, 6 R n^2 entries over
    n^3 points)."""
    b = 2 * csz + rsz
    if first:
        b += 32.0 * 6 * R / n
    return b


def launch_step_share(label):
    """Fraction of one step's grid-point updates a launch performs: a launch
    of the one-pass sweep carries the whole step, a two-stage half one half, a
    stage of the staged sweep one quarter.  Face-only launches update no grid
    points (None)."""
    if label == "fused_step":
        return 1.0
    if label.startswith("fused2_half"):
        return 0.5
    if label.startswith("stage_"):
        return 0.25
    return None


def launch_io_bytes(label, n, R, csz, rsz, first=True):
    """Bytes a launch itself reads and writes once at n^3 (state csz,
    potential rsz, FP64 face aux 16 B): the implementation's own traffic,
    which counts the intermediate stage arrays the method does not need."""
    npts = n ** 3
    faces = 6 * R * n * n
    if label == "fused_step":
        return npts * (2 * csz + rsz) + (faces * 32 if first else 0)
    if label == "fused2_half_a":                    # read psi, V, f; write u2 and its aux
        return npts * (2 * csz + rsz) + (faces * 32 if first else 0)
    if label == "fused2_half_b":                    # read u2, psi, V, both aux; write psi', f'
        return npts * (3 * csz + rsz) + (faces * 48 if first else 0)
    if label in ("stage_1", "stage_3"):             # y in, V; z out
        return npts * (2 * csz + rsz)
    if label == "stage_2":                          # y in, psi, V; running sum and z out
        return npts * (4 * csz + rsz)
    if label == "stage_4":                          # y in, running sum, V; psi' out
        return npts * (3 * csz + rsz)
    if label.startswith("boundary_"):
        return faces * (16 * 3 + csz)
    return None


def roofline(table, n, R, csz, rsz, ms_step, traffic, first=True):
    """Roofline of the dominant grid sweep: its algorithmic bytes (the method's
    bytes per update times the updates the launch performs) over its average
    duration, against the 8 TB/s HBM peak.  impl_frac prices the same launch
    at its own I/O instead; traffic_ratio is the counted HBM bytes over the
    algorithmic bytes."""
    b_upd = method_bytes_per_update(n, R, csz, rsz, first)
    sweeps = [r for r in table if launch_step_share(r["launch"]) is not None and r["ms"] > 0]
    dom = max(sweeps or table, key=lambda r: r["ms"])
    share = launch_step_share(dom["launch"])
    alg = b_upd * n ** 3 * share if share else None
    achieved = alg / (dom["ms"] / 1e3) / 1e9 if alg else None
    io = launch_io_bytes(dom["launch"], n, R, csz, rsz, first)
    step_alg = b_upd * n ** 3
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic, "kernel": dom["launch"], "alg_bytes_per_update": b_upd,
            "step_share_per_launch": share, "alg_bytes_per_launch": alg, "avg_launch_ms": dom["ms"],
            "impl_bytes_per_launch": io,
            "impl_frac": (io / (dom["ms"] / 1e3) / 1e9 / HBM_PEAK_GBS) if io else None,
            "traffic_ratio": (traffic / alg) if (traffic and alg) else None,
            "step_alg_bytes": step_alg,
            "step_frac": step_alg / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
            "launches": table}


def measured_traffic(label, args):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, if it was taken on this launch, workload and the current kernel
    source; None otherwise."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s_%d_%s.txt" % (label, args.n, args.dtype))
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_1908_02456_amd", "csrc", fields.get("source", "fused.hip"))
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if fields.get("source_sha256") != sha:
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _time(torch, fn, stream=None):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def bench_c64(Solver, torch, wl, args, steps):
    """The headline workload with the complex64 stencil (FP64 aux), built from
    the same arguments as the headline (radius, window, taper, path): time per
    step, and its relative deviation from the complex128 run of the same
    problem after the workload's full step count."""
    kw = dict(radius=wl.radius, order="first", s1=wl.s1, window=args.window, fejer=not args.no_fejer,
              path=args.path)
    s = Solver((wl.n,) * 3, wl.h, wl.dt, dtype="c64", **kw)
    V32 = torch.from_numpy(wl.V).to(torch.float32).cuda()
    psi = torch.from_numpy(wl.psi0).to(torch.complex64).cuda()
    aux = s.new_aux()
    s.step(psi, aux, V32, 20)
    ms = _time(torch, lambda: s.step(psi, aux, V32, steps))
    psi = torch.from_numpy(wl.psi0).to(torch.complex64).cuda()
    aux = s.new_aux()
    s.step(psi, aux, V32, wl.steps)
    s128 = Solver((wl.n,) * 3, wl.h, wl.dt, dtype="c128", **kw)
    ref = torch.from_numpy(wl.psi0).cuda()
    s128.step(ref, s128.new_aux(), torch.from_numpy(wl.V).cuda(), wl.steps)
    torch.cuda.synchronize()
    d = psi.to(torch.complex128) - ref
    return {"ms_per_step": ms / steps, "value": wl.n ** 3 * steps / (ms / 1e3), "unit": "grid-point-updates/s",
            "rel_err_vs_c128_max": d.abs().max().item() / ref.abs().max().item(),
            "rel_err_vs_c128_l2": torch.linalg.vector_norm(d).item() / torch.linalg.vector_norm(ref).item(),
            "compared_after_steps": wl.steps}


def bench_batch(Batch, Solver, torch, W, steps=20):
    """64 uneven instances (N in {48..160}, mixed zeroth/first, complex128):
    tuned descriptor-driven launches, eager and graph-captured, against the
    same instances stepped one after another."""
    insts = W.uneven_batch()
    cfgs = [dict(shape=d["shape"], h=d["h"], dt=d["dt"], order=d["order"], s0=d["s0"], s1=d["s1"], window=0)
            for d in insts]
    b = Batch(cfgs)
    psis = [torch.from_numpy(d["psi0"]).cuda() for d in insts]
    Vs = [torch.from_numpy(d["V"]).cuda() for d in insts]
    auxs = [b.new_aux(i) for i in range(len(insts))]
    depths = b.tune(psis, auxs, Vs)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    pts = sum(int(np.prod(d["shape"])) for d in insts)
    with torch.cuda.stream(stream):
        b.step(psis, auxs, Vs, 2, stream=stream)
        ms_eager = _time(torch, lambda: b.step(psis, auxs, Vs, steps, stream=stream), stream)
        b.step(psis, auxs, Vs, steps, graph=True, stream=stream)
        ms_graph = _time(torch, lambda: b.step(psis, auxs, Vs, steps, graph=True, stream=stream), stream)
    singles = [Solver(d["shape"], d["h"], d["dt"], order=d["order"], s0=1.0, s1=1.0, window=0) for d in insts]
    saux = [s.new_aux() for s in singles]

    def seq():
        for s, p, a, v in zip(singles, psis, saux, Vs):
            s.step(p, a, v, steps)
    seq()
    ms_seq = _time(torch, seq)
    return {"instances": len(insts), "grid_points": pts, "steps": steps, "tile_depths": depths,
            "value_graph": pts * steps / (ms_graph / 1e3), "value_eager": pts * steps / (ms_eager / 1e3),
            "value_sequential_single": pts * steps / (ms_seq / 1e3), "unit": "grid-point-updates/s",
            "speedup_vs_sequential": ms_seq / ms_graph}


def bench_adjoint(Solver, torch, W):
    """Adjoint workload (96^3, 500 steps, first order, FP64): reverse-mode
    gradient with sqrt(n) checkpoints, and with the whole run kept as one
    segment, against the plain forward run."""
    prm = W.adjoint_packet()
    n = prm["n"]
    s = Solver((n,) * 3, prm["h"], prm["dt"], order="first", s1=prm["s1"], window=prm["window"])
    psi0 = torch.from_numpy(W.gaussian_packet((n,) * 3, prm["h"], center=prm["packet_center"], k=prm["k"])).cuda()
    V = torch.from_numpy(W.gaussian_well((n,) * 3, prm["h"], prm["amplitude"])).cuda()
    out = {}
    ms_adj = _time(torch, lambda: out.setdefault("r", s.adjoint(psi0, V, prm["steps"], "prob")))
    # one segment kept whole (every state and stage vector in HBM, about
    # 28 GB here): no recompute and no separate forward sweep
    ms_all = _time(torch, lambda: out.setdefault("a", s.adjoint(psi0, V, prm["steps"], "prob",
                                                                ckpt_stride=prm["steps"])))
    psi = psi0.clone()
    aux = s.new_aux()
    ms_fwd = _time(torch, lambda: s.step(psi, aux, V, prm["steps"]))
    dg = (out["r"][1] - out["a"][1]).abs().max().item() / out["r"][1].abs().max().item()
    return {"grid": n, "steps": prm["steps"], "J": out["r"][0], "ms_adjoint": ms_adj, "ms_forward": ms_fwd,
            "adjoint_over_forward": ms_adj / ms_fwd, "forward_path": s.path,
            "ms_adjoint_one_segment": ms_all, "one_segment_over_forward": ms_all / ms_fwd,
            "grad_psi0_rel_diff_between_the_two": dg}


def bench_tdhf(Solver, torch, W, steps=10, full_steps=1000):
    """32 oscillator orbitals on 96^3 with the mean field U = -rho + 0.5 rho^2,
    first-order condition, complex64 stencil / FP64 aux: time per step, and
    the relative deviation of the orbitals from the complex128 run of the same
    batch after the workload's 1000 steps."""
    n, nb, h = 96, 32, 0.2
    orb = W.oscillator_orbitals((n,) * 3, h, nb, seed=3)
    kw = dict(order="first", s1=1.0, window=0, batch=nb, meanfield=(-1.0, 0.5))
    s = Solver((n,) * 3, h, 0.002, dtype="c64", **kw)
    psi = torch.from_numpy(orb).to(torch.complex64).cuda().contiguous()
    aux = s.new_aux()
    s.step(psi, aux, None, 2)
    ms = _time(torch, lambda: s.step(psi, aux, None, steps))
    out = {"grid": n, "orbitals": nb, "steps": steps, "ms_per_step": ms / steps,
           "value": n ** 3 * nb * steps / (ms / 1e3), "unit": "orbital-point-updates/s",
           "path": ("orbital batch, " + s.path) if s.use_fused else "staged"}
    psi = torch.from_numpy(orb).to(torch.complex64).cuda().contiguous()
    aux = s.new_aux()
    s.step(psi, aux, None, full_steps)
    s128 = Solver((n,) * 3, h, 0.002, dtype="c128", **kw)
    ref = torch.from_numpy(orb).cuda().contiguous()
    ms128 = _time(torch, lambda: s128.step(ref, s128.new_aux(), None, full_steps))
    d = psi.to(torch.complex128) - ref
    out.update({"rel_err_vs_c128_max": d.abs().max().item() / ref.abs().max().item(),
                "rel_err_vs_c128_l2": torch.linalg.vector_norm(d).item() / torch.linalg.vector_norm(ref).item(),
                "compared_after_steps": full_steps, "c128_ms_per_step": ms128 / full_steps})
    return out


def bench_tdhf_skyrme(Solver, torch, W, steps=10):
    """The TDHF batch with the long-range terms of Sec. 4.3: every step first
    solves the Yukawa (range 0.7) and Coulomb fields of rho by conjugate
    gradients (relative residual 1e-12, warm-started), then steps the 32
    orbitals; time per step and iterations per solve."""
    n, nb, h = 96, 32, 0.2
    orb = W.oscillator_orbitals((n,) * 3, h, nb, seed=3)
    mf = dict(t0=-1.0, t3=0.5, v0=-0.5, a=0.7, e2=0.1, tol=1e-12, maxit=2000)
    s = Solver((n,) * 3, h, 0.002, order="first", s1=1.0, window=0, dtype="c64", batch=nb, meanfield=mf)
    psi = torch.from_numpy(orb).to(torch.complex64).cuda().contiguous()
    aux = s.new_aux()
    s.step(psi, aux, None, 2)
    e0, y0, c0 = s.potential_iterations()
    ms = _time(torch, lambda: s.step(psi, aux, None, steps))
    e1, y1, c1 = s.potential_iterations()
    out = {"grid": n, "orbitals": nb, "steps": steps, "ms_per_step": ms / steps,
           "value": n ** 3 * nb * steps / (ms / 1e3), "unit": "orbital-point-updates/s",
           "cg_iterations_per_step": {"yukawa": (y1 - y0) / (e1 - e0), "coulomb": (c1 - c0) / (e1 - e0)},
           "cold_start_iterations": {"yukawa": y0 / max(e0, 1), "coulomb": c0 / max(e0, 1)},
           "path": ("orbital batch, " + s.path) if s.use_fused else "staged"}
    # one CG iteration per solve issued without host reads (the sine-transform
    # preconditioner is exact at R = 1; the unconverged count checks it),
    # eagerly and as a captured graph of the same steps replayed
    del s
    fixed = 1
    sf = Solver((n,) * 3, h, 0.002, order="first", s1=1.0, window=0, dtype="c64", batch=nb,
                meanfield=dict(mf, fixed_iters=fixed))
    psi = torch.from_numpy(orb).to(torch.complex64).cuda().contiguous()
    aux = sf.new_aux()
    sf.step(psi, aux, None, 2)
    ms_fixed = _time(torch, lambda: sf.step(psi, aux, None, steps))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sf.step(psi, aux, None, steps)
    g.replay()
    ms_graph = _time(torch, lambda: g.replay())
    out["fixed_iterations"] = {"iterations_per_solve": fixed, "ms_per_step": ms_fixed / steps,
                               "ms_per_step_graph_replay": ms_graph / steps,
                               "value_graph_replay": n ** 3 * nb * steps / (ms_graph / 1e3),
                               "unconverged_solves": sf.potential_unconverged()}
    return out


def bench_r3(Solver, torch, wl, steps=20):
    """The same 128^3 first-order workload with the seven-points-per-axis
    stencil (R = 3), which runs on the general staged path."""
    s = Solver((wl.n,) * 3, wl.h, wl.dt, radius=3, order="first", s1=wl.s1, window=wl.window)
    psi = torch.from_numpy(wl.psi0).cuda()
    V = torch.from_numpy(wl.V).cuda()
    aux = s.new_aux()
    s.step(psi, aux, V, 2)
    ms = _time(torch, lambda: s.step(psi, aux, V, steps))
    return {"radius": 3, "ms_per_step": ms / steps, "value": wl.n ** 3 * steps / (ms / 1e3),
            "unit": "grid-point-updates/s", "path": s.path}


def bench_free_packet(Solver, torch, W, big=128):
    """The free-packet workload (32^3, h = 0.25, zeroth order s0 = 1, 200
    steps of dt = 0.005, k = 2 along x, centred) against the same packet in a
    big^3 zero-boundary box cut back to the small one: relative L2 error at
    T and time per step, for the dense box form (R = 1, and R = 3 against an
    R = 3 reference), the face form and zero boundary values."""
    wl = W.free_packet_small()
    n = wl.n
    off = (big - n) // 2
    refs = {}
    for R in (1, 3):
        pb = torch.zeros((big,) * 3, dtype=torch.complex128, device="cuda")
        pb[off:off + n, off:off + n, off:off + n] = torch.from_numpy(wl.psi0).cuda()
        Solver((big,) * 3, wl.h, wl.dt, order="dirichlet", radius=R).step(pb, None, None, wl.steps)
        refs[R] = pb[off:off + n, off:off + n, off:off + n].clone()
        del pb
    out = {"grid": n, "reference_grid": big, "h": wl.h, "dt": wl.dt, "steps": wl.steps, "T": wl.steps * wl.dt}
    for name, kw in (("zeroth_box", dict(order="zeroth", form="box", s0=wl.s0)),
                     ("zeroth_box_R3", dict(order="zeroth", form="box", s0=wl.s0, radius=3)),
                     ("zeroth_faces", dict(order="zeroth", form="faces", s0=wl.s0)),
                     ("dirichlet", dict(order="dirichlet"))):
        s = Solver((n,) * 3, wl.h, wl.dt, **kw)
        psi = torch.from_numpy(wl.psi0).cuda().contiguous()
        s.step(psi, None, None, wl.steps)
        torch.cuda.synchronize()
        ref = refs[kw.get("radius", 1)]
        e = torch.linalg.vector_norm(psi - ref).item() / torch.linalg.vector_norm(ref).item()
        ms = _time(torch, lambda: s.step(psi, None, None, 50)) / 50
        out[name] = {"err_vs_large_box": e, "ms_per_step": ms, "path": s.path}
        del s, psi
        torch.cuda.empty_cache()
    return out


def bench_box_batch(Solver, torch, W, nb=32, steps=20):
    """Paper-literal dense box form (32^3, R = 1, zeroth order, free packet)
    over an orbital batch: one complex GEMM per stage for all orbitals,
    against the single-orbital GEMV path run once per orbital."""
    wl = W.free_packet_small()
    n = wl.n
    psi1 = torch.from_numpy(wl.psi0).cuda()
    s1 = Solver((n,) * 3, wl.h, wl.dt, order="zeroth", form="box", s0=wl.s0)
    s1.step(psi1, None, None, 2)
    ms1 = _time(torch, lambda: s1.step(psi1, None, None, steps))
    sb = Solver((n,) * 3, wl.h, wl.dt, order="zeroth", form="box", s0=wl.s0, batch=nb)
    psib = psi1.unsqueeze(-1).repeat(1, 1, 1, nb).contiguous()
    sb.step(psib, None, None, 2)
    msb = _time(torch, lambda: sb.step(psib, None, None, steps))
    return {"grid": n, "orbitals": nb, "value_gemm_batch": n ** 3 * nb * steps / (msb / 1e3),
            "value_single_orbital": n ** 3 * steps / (ms1 / 1e3), "unit": "orbital-point-updates/s",
            "speedup_vs_per_orbital": (ms1 * nb) / msb}


def bench_orders_box(Solver, torch, W, n=16, big=40, h=0.25, dt=0.005, steps=200):
    """The dense box form with each order on a free packet (k = 2 along x)
    leaving an n^3 box: relative L2 error at T against a big^3 zero-boundary
    box (data zero-extended) and the time per step of each order."""
    psi0 = W.gaussian_packet((n,) * 3, h, k=(2.0, 0.0, 0.0))
    off = (big - n) // 2
    pb = torch.zeros((big,) * 3, dtype=torch.complex128, device="cuda")
    pb[off:off + n, off:off + n, off:off + n] = torch.from_numpy(psi0).cuda()
    Solver((big,) * 3, h, dt, order="dirichlet").step(pb, None, None, steps)
    ref = pb[off:off + n, off:off + n, off:off + n].clone()
    nr = torch.linalg.vector_norm(ref).item()
    out = {"grid": n, "reference_grid": big, "h": h, "dt": dt, "steps": steps, "T": steps * dt}
    for name, kw in (("dirichlet", dict(order="dirichlet")), ("zeroth", dict(order="zeroth", s0=1.0)),
                     ("first", dict(order="first", s1=1.0)), ("first_two_point", dict(order="first", s1=1.0, s2=4.0)),
                     ("second", dict(order="second", s_points=(1.0, 2.0, 3.0, 10.0)))):
        t0 = time.perf_counter()
        s = Solver((n,) * 3, h, dt, form="box", **kw)
        setup_s = time.perf_counter() - t0
        psi = torch.from_numpy(psi0).cuda()
        aux = s.new_aux()
        s.step(psi, aux, None, steps)
        torch.cuda.synchronize()
        e = torch.linalg.vector_norm(psi - ref).item() / nr
        p2 = torch.from_numpy(psi0).cuda()
        a2 = s.new_aux()
        s.step(p2, a2, None, 2)
        ms = _time(torch, lambda: s.step(p2, a2, None, 20)) / 20
        out[name] = {"err_vs_large_box": e, "ms_per_step": ms, "setup_s": setup_s}
    return out


def bench_box64(Solver, torch, W, n=64, big=128, h=0.25, dt=0.005, steps=500):
    """Face form against the paper's dense box form on a 64^3 box
    (n_Gamma = 23816; the box operators are built on the device): a free
    packet exp(-|x - (4, 0, 0)|^2/2) e^{2ix} leaving the box, relative L2
    error at T against a 128^3 zero-boundary box (data zero-extended), with
    setup time and time per step."""
    psi0 = W.gaussian_packet((n,) * 3, h, center=(4.0, 0.0, 0.0), k=(2.0, 0.0, 0.0))
    off = (big - n) // 2
    pb = torch.zeros((big,) * 3, dtype=torch.complex128, device="cuda")
    pb[off:off + n, off:off + n, off:off + n] = torch.from_numpy(psi0).cuda()
    Solver((big,) * 3, h, dt, order="dirichlet").step(pb, None, None, steps)
    ref = pb[off:off + n, off:off + n, off:off + n].clone()
    del pb
    nr = torch.linalg.vector_norm(ref).item()
    out = {"grid": n, "reference_grid": big, "h": h, "dt": dt, "steps": steps, "T": steps * dt}
    for name, kw in (("dirichlet", dict(order="dirichlet")),
                     ("faces_first_w0", dict(order="first", s1=1.0, window=0)),
                     ("faces_first_w8", dict(order="first", s1=1.0, window=8)),
                     ("box_zeroth", dict(order="zeroth", s0=1.0, form="box")),
                     ("box_first", dict(order="first", s1=1.0, form="box"))):
        log("  box64: %s" % name)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = Solver((n,) * 3, h, dt, **kw)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        psi = torch.from_numpy(psi0).cuda()
        aux = s.new_aux()
        ms = _time(torch, lambda: s.step(psi, aux, None, steps)) / steps
        e = torch.linalg.vector_norm(psi - ref).item() / nr
        out[name] = {"err_vs_large_box": e, "ms_per_step": ms, "setup_s": setup_s,
                     "device_bytes": s.device_bytes()}
        del s, psi, aux
        torch.cuda.empty_cache()
    return out


def bench_h2_point(Solver, torch, wl, modes=64, nodes=4096):
    """The H2-optimal first-order point (Sec. 5 proposal) of the face form at
    the headline h for windows 0 and 8: time per objective evaluation on the
    device, the minimiser, and the physics error of the headline run (2000
    steps, 128^3) at that point against s1 = 1.  (The oracle's time for the
    same objective is part of the CPU baseline.)"""
    from paper_1908_02456_amd import solver as api
    pts = np.exp(np.linspace(math.log(0.1), math.log(1000.0), 8))
    api.h2_objective(wl.h, pts[:1], modes=modes, nodes=nodes)
    t0 = time.perf_counter()
    api.h2_objective(wl.h, pts, modes=modes, nodes=nodes)
    gpu_s = (time.perf_counter() - t0) / len(pts)
    out = {"modes": modes, "nodes": nodes, "gpu_s_per_point": gpu_s,
           "gpu_integrand_evals_per_s": modes * modes * nodes / gpu_s}
    ref = large_box_reference(Solver, torch, wl, "auto", wl.steps)
    nr = torch.linalg.vector_norm(ref).item()
    V = torch.from_numpy(wl.V).cuda()
    for w in (0, 8):
        s_best, j_best = api.optimal_point(wl.h, window=w, modes=modes, nodes=nodes)
        row = {"s1_opt": s_best, "J_opt": j_best,
               "J_at_1": float(api.h2_objective(wl.h, 1.0, window=w, modes=modes, nodes=nodes)[0])}
        for tag, s1 in (("s1_1", 1.0), ("s1_opt", s_best)):
            s = Solver((wl.n,) * 3, wl.h, wl.dt, order="first", s1=s1, window=w)
            psi = torch.from_numpy(wl.psi0).cuda()
            aux = s.new_aux()
            s.step(psi, aux, V, wl.steps)
            torch.cuda.synchronize()
            row["err_" + tag] = torch.linalg.vector_norm(psi - ref).item() / nr
        out["w%d" % w] = row
    return out


def bench_face_windows(Solver, torch, wl, steps_timed=20):
    """The headline workload with wider face operators: w = 0 (one-pass
    sweep), w = 8 with the Fejer window (direct convolution) and the exact
    section w = n - 1 (zero-padded 2D FFTs), the wider two on the staged path
    and on the one-pass sweep with boundary-shell rounds: time per step and
    the relative error against the large zero-boundary box after 2000 steps."""
    ref = large_box_reference(Solver, torch, wl, "auto", wl.steps)
    nr = torch.linalg.vector_norm(ref).item()
    V = torch.from_numpy(wl.V).cuda()
    out = {}
    for name, w, fejer, path in (("w0", 0, True, "auto"), ("w8_fejer", 8, True, "auto"),
                                 ("w8_fejer_onepass", 8, True, "onepass"),
                                 ("exact_fft", wl.n - 1, False, "auto"),
                                 ("exact_fft_onepass", wl.n - 1, False, "onepass")):
        log("  face windows: %s" % name)
        s = Solver((wl.n,) * 3, wl.h, wl.dt, order="first", s1=wl.s1, window=w, fejer=fejer, path=path)
        psi = torch.from_numpy(wl.psi0).cuda()
        aux = s.new_aux()
        s.step(psi, aux, V, 2)
        ms = _time(torch, lambda: s.step(psi, aux, V, steps_timed)) / steps_timed
        psi = torch.from_numpy(wl.psi0).cuda()
        aux = s.new_aux()
        s.step(psi, aux, V, wl.steps)
        torch.cuda.synchronize()
        out[name] = {"window": w, "fejer": fejer, "ms_per_step": ms, "path": s.path,
                     "err_vs_large_box": torch.linalg.vector_norm(psi - ref).item() / nr}
        del s, psi, aux
        torch.cuda.empty_cache()
    return out


def bench_paper_replica(Solver, torch, W, steps=600, every=50, big=97):
    """The paper's 3D experiment (Sec. 4.2) at its own size: box [-1.5, 1.5]^3,
    h = 0.1 (31^3 points), seven-point-per-axis stencil (R = 3, n_Gamma =
    14166), psi0 = exp(-|x|^2 + 5 i x1), dt = 0.001, dense box-form operators
    built on the device: first order from s = 1, 2 and second order from
    s = 1, 2, 3, 10.  Records the probability in the box every `every` steps
    for zero boundary values, both ABCs and a big^3 zero-boundary box cut back
    to the small one (reflections from its walls cannot return in time), and
    the relative L2 error of each run against that reference."""
    n, h, dt, R = 31, 0.1, 0.001, 3
    x = (np.arange(n) - (n - 1) / 2) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    psi0 = np.exp(-(X ** 2 + Y ** 2 + Z ** 2) + 5j * X)
    off = (big - n) // 2
    norm0 = float(np.linalg.norm(psi0))
    out = {"grid": n, "h": h, "dt": dt, "radius": R, "steps": steps, "reference_grid": big}
    pb = torch.zeros((big,) * 3, dtype=torch.complex128, device="cuda")
    pb[off:off + n, off:off + n, off:off + n] = torch.from_numpy(psi0).cuda()
    sb = Solver((big,) * 3, h, dt, radius=R, order="dirichlet")
    refs, nref = [], []
    for k in range(steps // every):
        sb.step(pb, None, None, every)
        inner = pb[off:off + n, off:off + n, off:off + n].clone()
        refs.append(inner)
        nref.append(h ** 3 * float(torch.sum(torch.abs(inner) ** 2)))
    out["norm_reference"] = nref
    del sb, pb
    for name, kw in (("dirichlet", dict(order="dirichlet")),
                     ("first_s12", dict(order="first", form="box", s1=1.0, s2=2.0)),
                     ("second_s12310", dict(order="second", form="box", s_points=(1.0, 2.0, 3.0, 10.0)))):
        log("  paper replica: %s" % name)
        t0 = time.perf_counter()
        try:
            s = Solver((n,) * 3, h, dt, radius=R, **kw)
        except Exception as exc:  # recorded: the setup's own stability check
            out[name] = {"setup_error": str(exc)}
            continue
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        psi = torch.from_numpy(psi0).cuda()
        aux = s.new_aux()
        norms, errs = [], []
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(steps // every):
            s.step(psi, aux, None, every)
            norms.append(h ** 3 * float(torch.sum(torch.abs(psi) ** 2)))
            errs.append(torch.linalg.vector_norm(psi - refs[k]).item() / norm0)
        e1.record()
        torch.cuda.synchronize()
        out[name] = {"setup_s": setup_s, "ms_per_step": e0.elapsed_time(e1) / steps, "norm": norms,
                     "err_vs_reference": errs, "device_bytes": s.device_bytes()}
        if kw.get("form") == "box":
            out[name].update(s.box_info())
        del s, psi, aux
        torch.cuda.empty_cache()
    return out


def cpu_baseline(wl, window, budget_s=15.0, fejer=True):
    """FP64 oracle (NumPy, single-threaded elementwise) on the same workload,
    for as many whole steps as fit in about budget_s seconds.  Returns the
    record and the oracle's state after those steps."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle import integrate
    st = integrate.make_setup((wl.n,) * 3, wl.h, wl.dt, wl.radius, "first", s1=wl.s1, window=window,
                              use_window=fejer)
    psi, aux = wl.psi0.copy(), integrate.zero_aux(st)
    ctx = threadpool_limits(1) if threadpool_limits else None
    if ctx:
        ctx.__enter__()
    try:
        t0 = time.perf_counter()
        steps = 0
        while True:
            psi, aux = integrate.taylor4_step(st, psi, aux, wl.V)
            steps += 1
            el = time.perf_counter() - t0
            if el > budget_s or steps >= 50:
                break
        # the oracle's H2 objective of the first-order point (one candidate)
        from oracle import h2
        t0 = time.perf_counter()
        h2.h2_objective(wl.h, 1.0, 0, P=32, N=1024)
        h2_s = time.perf_counter() - t0
    finally:
        if ctx:
            ctx.__exit__(None, None, None)
    rec = {"value": wl.n ** 3 * steps / el, "unit": "grid-point-updates/s", "cores": 1, "kind": "oracle",
           "sample": "%d Taylor steps of the same %d^3 first-order face-form workload (FP64 NumPy, %.1f s)"
                     % (steps, wl.n, el),
           "h2_objective": {"s_per_point": h2_s, "integrand_evals_per_s": 32 * 32 * 1024 / h2_s,
                            "sample": "one candidate, 32 x 32 modes x 1024 nodes"}}
    return rec, psi, steps


def errors_vs_oracle(Solver, torch, wl, args, psi_oracle, steps):
    """Relative error of the device runs in both precisions against the
    oracle's state after the same steps of the headline problem (the oracle's
    sample above)."""
    kw = dict(radius=wl.radius, order="first", s1=wl.s1, window=args.window, fejer=not args.no_fejer,
              path=args.path)
    ref = torch.from_numpy(psi_oracle)
    out = {"steps": steps}
    for dt_name, cdt, rdt in (("c128", torch.complex128, torch.float64), ("c64", torch.complex64, torch.float32)):
        s = Solver((wl.n,) * 3, wl.h, wl.dt, dtype=dt_name, **kw)
        psi = torch.from_numpy(wl.psi0).to(cdt).cuda()
        s.step(psi, s.new_aux(), torch.from_numpy(wl.V).to(rdt).cuda(), steps)
        torch.cuda.synchronize()
        d = psi.cpu().to(torch.complex128) - ref
        out[dt_name] = {"rel_err_max": d.abs().max().item() / ref.abs().max().item(),
                        "rel_err_l2": torch.linalg.vector_norm(d).item() / torch.linalg.vector_norm(ref).item()}
    return out


def tdhf_oracle_sample(Solver, torch, W, steps=1):
    """The TDHF batch (96^3, 32 orbitals, t0/t3 mean field, first order) in the
    oracle for one step (about 17 s on one core): its time per step, and the complex64
    device run's relative error against it after the same steps."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle import integrate
    n, nb, h, dt = 96, 32, 0.2, 0.002
    orb = W.oscillator_orbitals((n,) * 3, h, nb, seed=3)
    st = integrate.make_setup((n,) * 3, h, dt, 1, "first", s1=1.0, window=0, t0=-1.0, t3=0.5)
    V0 = np.zeros((n,) * 3)
    ctx = threadpool_limits(1) if threadpool_limits else None
    if ctx:
        ctx.__enter__()
    try:
        t0 = time.perf_counter()
        psi, aux = orb.copy(), integrate.zero_aux(st, nb)
        for _ in range(steps):
            psi, aux = integrate.taylor4_step(st, psi, aux, V0)
        el = time.perf_counter() - t0
    finally:
        if ctx:
            ctx.__exit__(None, None, None)
    s = Solver((n,) * 3, h, dt, order="first", s1=1.0, window=0, dtype="c64", batch=nb, meanfield=(-1.0, 0.5))
    g = torch.from_numpy(orb).to(torch.complex64).cuda().contiguous()
    s.step(g, s.new_aux(), None, steps)
    torch.cuda.synchronize()
    ref = torch.from_numpy(psi)
    d = g.cpu().to(torch.complex128) - ref
    return {"steps": steps, "oracle_s_per_step": el / steps,
            "oracle_orbital_point_updates_per_s": n ** 3 * nb * steps / el, "cores": 1,
            "c64_rel_err_max": d.abs().max().item() / ref.abs().max().item(),
            "c64_rel_err_l2": torch.linalg.vector_norm(d).item() / torch.linalg.vector_norm(ref).item()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--window", type=int, default=0)
    ap.add_argument("--radius", type=int, default=1, choices=[1, 2, 3], help="stencil half-width R")
    ap.add_argument("--no-fejer", action="store_true",
                    help="face kernels truncated without the triangular taper (w >= n - 1: exact sections)")
    ap.add_argument("--path", default="auto", choices=["auto", "staged", "fused", "onepass"])
    ap.add_argument("--no-physics", action="store_true")
    ap.add_argument("--replica", action="store_true",
                    help="also run the paper's 3D experiment at its own size (31^3, R = 3, dense box operators)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the batch / adjoint / c64 / TDHF figures")
    ap.add_argument("--only-extra", default="",
                    help="comma-separated names: run only these of the extra figures (e.g. tdhf,batch)")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="also run one plain device copy of this size (calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the stepper has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_02456_amd import workloads as W
    from paper_1908_02456_amd.solver import Solver

    wl = W.well_packet(n=args.n, window=args.window, radius=args.radius)
    cdt = torch.complex128 if args.dtype == "c128" else torch.complex64
    rdt = torch.float64 if args.dtype == "c128" else torch.float32
    log("setup: %d^3 first-order faces R=%d w=%d%s %s path=%s" % (wl.n, wl.radius, args.window,
                                                              " (no taper)" if args.no_fejer else "",
                                                              args.dtype, args.path))
    s = Solver((wl.n,) * 3, wl.h, wl.dt, radius=wl.radius, order="first", s1=wl.s1, window=args.window,
               fejer=not args.no_fejer, dtype=args.dtype, path=args.path)
    psi = torch.from_numpy(wl.psi0).to(cdt).cuda().contiguous()
    V = torch.from_numpy(wl.V).to(rdt).cuda().contiguous()
    aux = s.new_aux()
    stream = torch.cuda.current_stream()
    s.step(psi, aux, V, args.warmup)
    torch.cuda.synchronize()
    log("warmup done (%d steps)" % args.warmup)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    s.step(psi, aux, V, args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ms_step = ms / args.steps
    npts = wl.n ** 3
    value = npts * args.steps / (ms / 1e3)
    log("timed %d steps: %.3f ms/step, %.3e GPUPS" % (args.steps, ms_step, value))

    # per-launch durations (HIP events around every launch, same stream), then
    # the roofline of the dominant launch from its algorithmic bytes
    per_launch = s.step_timed(psi, aux, V, args.steps, stream=stream)
    torch.cuda.synchronize()
    csz = 16 if args.dtype == "c128" else 8
    rsz = 8 if args.dtype == "c128" else 4
    table = []
    for label, lms in per_launch:
        b = launch_io_bytes(label, wl.n, wl.radius, csz, rsz)
        table.append({"launch": label, "ms": lms, "impl_bytes": b,
                      "impl_GB/s": (b / (lms / 1e3) / 1e9) if (b and lms > 0) else None})
    log("launches per step: " + ", ".join("%s %.2f us" % (r["launch"], r["ms"] * 1e3) for r in table))
    sweeps = [r["launch"] for r in table if launch_step_share(r["launch"]) is not None]
    dom_label = max((r for r in table if r["launch"] in sweeps), key=lambda r: r["ms"])["launch"] if sweeps else None
    roof = roofline(table, wl.n, wl.radius, csz, rsz, ms_step,
                    measured_traffic(dom_label, args) if dom_label else None)

    out = {"metric": "grid-point-updates/s incl. ABC (% HBM roofline); err vs FP64 large-box oracle",
           "value": value, "unit": "grid-point-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if args.dtype == "c128" else "f32 stencil / f64 aux",
           "data": "synthetic",
           "config": {"workload": "single orbital %d^3, h=%.2g, dt=%.3g, first-order face-form DtN ABC "
                                  "(s1=%.3g, w=%d), Gaussian well + k=(3,1,0) packet, %s"
                                  % (wl.n, wl.h, wl.dt, wl.s1, args.window, args.dtype),
                      "grid": [wl.n] * 3, "radius": wl.radius, "fejer": not args.no_fejer, "path": args.path,
                      "path_chosen": s.path},
           "roofline": roof}
    if args.copy_gib > 0:
        nb = int(args.copy_gib * (1 << 30)) // 16 * 16
        src_t = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * nb
        del src_t, dst_t
    only = set(v for v in args.only_extra.split(",") if v)
    if not args.no_extra:
        from paper_1908_02456_amd.solver import Batch
        extra = {}
        for name, fn in (("c64", lambda: bench_c64(Solver, torch, wl, args, 200)),
                         ("batch", lambda: bench_batch(Batch, Solver, torch, W)),
                         ("adjoint", lambda: bench_adjoint(Solver, torch, W)),
                         ("tdhf", lambda: bench_tdhf(Solver, torch, W)),
                         ("tdhf_skyrme", lambda: bench_tdhf_skyrme(Solver, torch, W)),
                         ("r3", lambda: bench_r3(Solver, torch, wl)),
                         ("free_packet", lambda: bench_free_packet(Solver, torch, W)),
                         ("box_batch", lambda: bench_box_batch(Solver, torch, W)),
                         ("orders_box", lambda: bench_orders_box(Solver, torch, W)),
                         ("box64", lambda: bench_box64(Solver, torch, W)),
                         ("h2_point", lambda: bench_h2_point(Solver, torch, wl)),
                         ("face_windows", lambda: bench_face_windows(Solver, torch, wl))):
            if only and name not in only:
                continue
            log("extra: %s" % name)
            try:
                extra[name] = fn()
            except Exception as exc:  # reported, not fatal for the headline line
                extra[name] = {"error": repr(exc)}
            torch.cuda.empty_cache()
        out["extra"] = extra
    if args.replica:
        log("paper replica (31^3, R = 3, box form)")
        out["paper_replica"] = bench_paper_replica(Solver, torch, W)
    if not args.no_physics:
        log("physics run: %d steps vs %d^3 zero-boundary box" % (wl.steps, 2 * wl.n))
        out["physics"] = physics_error(Solver, torch, wl, args.dtype, args.window, args.path, wl.steps,
                                       fejer=not args.no_fejer)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cb, psi_or, k = cpu_baseline(wl, args.window, fejer=not args.no_fejer)
        cb["errors_vs_oracle"] = errors_vs_oracle(Solver, torch, wl, args, psi_or, k)
        if not args.no_extra:
            log("cpu baseline: TDHF oracle sample ...")
            cb["tdhf_sample"] = tdhf_oracle_sample(Solver, torch, W)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
