"""Benchmark of the fused D2Q9 TRT-VP step on one MI355X.

One step = one pass of the whole hot path over the large single domain
(8192 x 4096 nodes, two counter-rotating cylinders, a tandem pair and a NACA-0012
airfoil, Re = 200, U = 0.04): the fused pull-stream / moments / penalization /
TRT-collision kernel plus the per-body force and global mass reduction of every
step. Inputs are synthetic and resident in HBM before timing starts.

Prints one JSON line: MLUPS (10^6 lattice-node updates per second, all nodes
counted), the HBM roofline fraction of the step kernel from algorithmic bytes
(9 loads + 9 stores + 1 mask byte per node) and HIP-event timing on the
solver's stream, and the FP64 CPU oracle timed on the host's cores on a bounded
sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage f32|f16|bf16|f64]
"""
import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "MLUPS + % of HBM peak, plain vs batched/FP16; p50/p99 solve latency"
# the nine populations read and written once per step in the storage type; the
# body-mask byte is added per node where the step reads it (alg_bytes_per_node)
POP_BYTES = {"f64": 144, "f32": 72, "f16": 36, "bf16": 36}
COUNTERS_FILE = os.path.join(ROOT, "profiles", "step_kernel_counters.json")
# per lattice: populations per node, the sources its step kernel is built from,
# and the committed counter summary of that kernel
LATTICES = {
    "d2q9": {"q": 9, "sources": ("lbvp_kernels.hip", "lbvp_device.h", "lbvp_internal.h"),
             "counters": COUNTERS_FILE},
    "d3q19": {"q": 19, "sources": ("lbvp3_kernels.hip", "lbvp_device.h", "lbvp3_internal.h"),
              "counters": os.path.join(ROOT, "profiles", "step3_kernel_counters.json")},
}
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


def kernel_source_hash(lattice: str = "d2q9") -> str:
    h = hashlib.sha256()
    for name in LATTICES[lattice]["sources"]:
        with open(os.path.join(ROOT, "paper_1901_08766_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(storage: str, nodes: int, lattice: str = "d2q9", key: str = None):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    try:
        with open(LATTICES[lattice]["counters"]) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_hash") != kernel_source_hash(lattice):
        return None
    entry = c.get("per_storage", {}).get(key or storage)
    if not entry or entry.get("nodes") != nodes:
        return None
    return entry.get("hbm_bytes_per_launch")


# the default D2Q9 launch of the 8192 x 4096 domain per storage type (the
# library's choice, which the GPU tests check)
DEFAULT_LAUNCH_2D = {"f32": {"vec": 4, "block": 128}, "f64": {"vec": 2, "block": 128},
                     "f16": {"vec": 4, "block": 256}, "bf16": {"vec": 4, "block": 256}}


def tile_shape(nx: int, launch, d3q19: bool = False) -> tuple:
    """(tile_w, tile_rows) of a launch shape (vec nodes per thread, block threads):
    on a narrow grid a D2Q9 tile row is nx rounded up to a power of two, a D3Q19
    one nx rounded up to vec."""
    vec, block = launch["vec"], launch["block"]
    if d3q19:
        tile_w = min(vec * block, -(-max(nx, 1) // vec) * vec)
    else:
        tile_w = min(vec * block, max(vec, 1 << max(nx - 1, 0).bit_length()))
    return tile_w, vec * block // tile_w


def mask_read_fraction(prob, launch) -> float:
    """Nodes whose mask byte a step reads, over all nodes: the nodes of tiles that
    hold a solid node (the step kernels skip the mask of every other tile). A 3-D
    mask [nz][ny][nx] is tiled as its nz ny lattice rows."""
    if prob.mask is None or not (prob.mask > 0).any():
        return 0.0
    mask = prob.mask.reshape(-1, prob.mask.shape[-1])
    ny, nx = mask.shape
    tw, tr = tile_shape(nx, launch, d3q19=prob.mask.ndim == 3)
    tx, ty = -(-nx // tw), -(-ny // tr)
    pad = np.zeros((ty * tr, tx * tw), dtype=bool)
    pad[:ny, :nx] = mask > 0
    has = pad.reshape(ty, tr, tx, tw).any(axis=(1, 3))
    w = np.minimum(tw, nx - np.arange(tx) * tw)            # real columns per tile column
    h = np.minimum(tr, ny - np.arange(ty) * tr)            # real rows per tile row
    return float((has * h[:, None] * w[None, :]).sum()) / (nx * ny)


def alg_bytes_per_node(storage: str, prob, launch) -> float:
    """Algorithmic HBM bytes per node of one step: 18 population accesses in the
    storage type plus the mask byte where the step reads it."""
    return POP_BYTES[storage] + mask_read_fraction(prob, launch)


def time_gpu(storage: str, steps: int, warmup: int, prob, repeats: int = 1):
    """ms per step of `steps` steps after `warmup` untimed ones (HIP events on the
    solver's stream); with repeats > 1 the timed run is repeated and the median
    taken (every repeat's time is returned too)."""
    import torch
    from paper_1901_08766_amd import lbvp

    solver = lbvp.Solver(prob, storage=storage, force_every=1, force_capacity=steps + warmup + 16)
    stream = solver.stream
    solver.step(warmup)
    solver.synchronize()
    solver.forces()
    if repeats > 1:
        # repeated (variant) timings start from steady clocks: the variant's
        # context set-up leaves the GPU idle, and it needs some milliseconds of
        # load to come back to its full clock
        for _ in range(4):
            solver.step(25)
            solver.forces()
    runs, ok = [], True
    for _ in range(repeats):
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        solver.step(steps)
        stop.record(stream)
        stop.synchronize()
        torch.cuda.synchronize()
        runs.append(start.elapsed_time(stop) / steps)
        forces, mass, _ = solver.forces()
        ok = ok and bool((mass == mass).all()) and len(mass) == steps
    launch = {"vec": solver.launch[0], "block": solver.launch[1], "tile_band": solver.tile_band}
    solver.close()
    torch.cuda.empty_cache()
    if repeats == 1:
        return runs[0], ok, launch
    return float(np.median(runs)), ok, launch, runs


POP_BYTES_3D = {"f64": 304, "f32": 152, "f16": 76, "bf16": 76}
# the default D3Q19 launch of the sphere domain per storage type
DEFAULT_LAUNCH_3D = {"f64": {"vec": 1, "block": 128}, "f32": {"vec": 1, "block": 256},
                     "f16": {"vec": 4, "block": 128}, "bf16": {"vec": 4, "block": 128}}


def alg_bytes_per_node3(storage: str, prob, launch) -> float:
    """D3Q19: 38 population accesses in the storage type plus the mask byte where
    the step reads it."""
    return POP_BYTES_3D[storage] + mask_read_fraction(prob, launch)


def time_d3q19(storages, steps: int, warmup: int):
    """The D3Q19 step on the 512 x 256 x 256 sphere domain (default launch, force
    and mass recorded every step), per storage type."""
    import torch
    from paper_1901_08766_amd import inputs3, lbvp3

    prob = inputs3.sphere()
    n = prob.n_nodes
    out = {"workload": f"flow past a sphere {prob.nx}x{prob.ny}x{prob.nz}, D={prob.l_ref:g}, Re=300, U=0.05",
           "nodes": n, "per_storage": {}}
    for st in storages:
        s = lbvp3.Solver3(prob, storage=st, force_every=1, force_capacity=steps + warmup + 16)
        s.step(warmup)
        s.synchronize()
        s.forces()
        ms = _timed(s.stream, lambda: s.step(steps)) / steps
        _, mass, _ = s.forces()
        bpn = alg_bytes_per_node3(st, prob, {"vec": s.launch[0], "block": s.launch[1]})
        gbps = bpn * n / (ms * 1e-3) / 1e9
        out["per_storage"][st] = {"launch": list(s.launch), "tile_band": s.tile_band, "ms_per_step": round(ms, 4),
                                  "alg_bytes_per_node": round(bpn, 3),
                                  "MLUPS": round(n / (ms * 1e-3) / 1e6, 1), "achieved_GBps": round(gbps, 1),
                                  "hbm_frac": round(gbps / HBM_PEAK_GBPS, 4),
                                  "traffic": measured_traffic(st, n, "d3q19"),
                                  "finite": bool(np.isfinite(mass).all() and len(mass) == steps)}
        print(f"# d3q19 {st}: {out['per_storage'][st]}", file=sys.stderr, flush=True)
        s.close()
        torch.cuda.empty_cache()
    return out


def time_ensemble3(storage: str, steps: int, n_dom: int = 64):
    """The D3Q19 ensemble of uneven sphere domains as one batch (one launch per
    step over all their tiles; launch shape and band from lbvp3_tune) against
    each domain's own launch per step, round-robin on one stream, at the same
    storage type."""
    import torch
    from paper_1901_08766_amd import inputs3, lbvp3

    probs = inputs3.ensemble3(n=n_dom)
    nodes = sum(p.n_nodes for p in probs)
    stream = torch.cuda.Stream()
    members = [lbvp3.Solver3(p, storage=storage, force_every=1, force_capacity=2 * steps + 64, stream=stream)
               for p in probs]
    out = {"workload": f"{n_dom} sphere domains, nx {inputs3.ENSEMBLE3_NX}, ny and nz {inputs3.ENSEMBLE3_NYZ}",
           "domains": n_dom, "nodes": nodes, "storage": storage}

    def drain():
        for m in members:
            m.forces()

    def per_domain():
        for _ in range(steps):
            for m in members:
                m.step(1)

    for m in members:
        m.step(2)
    drain()
    ms = _timed(stream, per_domain)
    out["per_domain_MLUPS"] = round(nodes * steps / ms / 1e3, 1)
    drain()
    # the stronger per-domain forms: captured graphs of `chunk` steps per domain,
    # and each domain's whole run as one call in turn
    chunk = min(20, steps)
    for m in members:
        m.step(chunk, graph=True)             # capture outside the timed region
    drain()
    ms = _timed(stream, lambda: [m.step(chunk, graph=True) for _ in range(steps // chunk) for m in members])
    out["per_domain_graph_MLUPS"] = round(nodes * (steps // chunk) * chunk / ms / 1e3, 1)
    drain()
    ms = _timed(stream, lambda: [m.step(steps) for m in members])
    out["per_domain_whole_run_MLUPS"] = round(nodes * steps / ms / 1e3, 1)
    drain()
    best_per_domain = max(out["per_domain_MLUPS"], out["per_domain_graph_MLUPS"], out["per_domain_whole_run_MLUPS"])
    rows, best = lbvp3.tune(members, steps=20)
    vec, block, band = best["vec"], best["block"], best["band"]
    out["tuner_rows"] = len(rows)
    batch = lbvp3.Batch3(members, vec, block)
    batch.set_tile_band(band)
    batch.step(5)
    drain()
    ms = _timed(stream, lambda: batch.step(steps))
    _, mass, _ = members[0].forces()
    drain()
    out.update({"launch": [vec, block], "tile_band": band, "batched_MLUPS": round(nodes * steps / ms / 1e3, 1),
                "batched_ms_per_step": round(ms / steps, 4),
                "speedup": round(nodes * steps / ms / 1e3 / max(out["per_domain_MLUPS"], 1e-9), 2),
                "speedup_vs_best_per_domain": round(nodes * steps / ms / 1e3 / max(best_per_domain, 1e-9), 2),
                "finite": bool(np.isfinite(mass).all())})
    batch.close()
    for m in members:
        m.close()
    torch.cuda.empty_cache()
    print(f"# d3q19 ensemble {storage}: {out}", file=sys.stderr, flush=True)
    return out


def time_slabs(n_slabs: int, steps: int = 100, storage: str = "f32"):
    """The large domain cut into n_slabs x-slabs on this one GPU (a halo exchange
    over every cut, then one batched step of all slabs) against the whole
    domain; and one slab alone, closed on itself through its own halo exchange:
    the share one GPU of n_slabs would step, with its exchange."""
    import torch
    from paper_1901_08766_amd import inputs, lbvp

    prob = inputs.large_domain()
    nodes = prob.nx * prob.ny
    w = prob.nx // n_slabs
    widths = [w] * (n_slabs - 1) + [prob.nx - w * (n_slabs - 1)]
    out = {"workload": f"large single domain {prob.nx}x{prob.ny} in {n_slabs} x-slabs of {w}", "storage": storage}
    whole = lbvp.Solver(prob, storage=storage, force_every=1, force_capacity=steps + 16)
    whole.step(5)
    whole.forces()
    out["whole_ms_per_step"] = round(_timed(whole.stream, lambda: whole.step(steps)) / steps, 4)
    whole.forces()
    whole.close()
    torch.cuda.empty_cache()
    slabs_p, x0s = inputs.split_x(prob, widths)
    slabs = lbvp.Slabs(slabs_p, x0s, storage=storage, force_every=1, force_capacity=steps + 16)
    slabs.step(5)
    slabs.forces()
    ms = _timed(slabs.stream, lambda: slabs.step(steps)) / steps
    slabs.forces()
    slabs.step(steps, graph=True)              # capture outside the timed region
    slabs.forces()
    msg = _timed(slabs.stream, lambda: slabs.step(steps, graph=True)) / steps
    slabs.forces()
    out["slabs_graph_ms_per_step"] = round(msg, 4)
    out["slabs_ms_per_step"] = round(ms, 4)
    out["slabs_MLUPS"] = round(nodes / (ms * 1e-3) / 1e6, 1)
    out["overhead_vs_whole"] = round(ms / out["whole_ms_per_step"] - 1.0, 4)
    ex = _timed(slabs.stream, lambda: [slabs.exchange() for _ in range(steps)]) / steps
    out["exchange_us_per_step"] = round(ex * 1e3, 2)
    out["bytes_per_cut_per_step"] = 2 * 3 * prob.ny * STORAGE_BYTES[storage]
    slabs.close()
    torch.cuda.empty_cache()
    # one slab, closed on itself: its halo exchange stands in for the transfer
    one = inputs.split_x(dataclasses.replace(prob, nx=w, bc=("periodic", "periodic", "periodic", "periodic"),
                                             mask=prob.mask[:, :w].copy(), rho_init=None, ux_init=None,
                                             uy_init=None), [w])[0]
    alone = lbvp.Slabs(one, [0], storage=storage, force_every=1, force_capacity=steps + 16)
    alone.step(5)
    alone.forces()
    ms1 = _timed(alone.stream, lambda: alone.step(steps)) / steps
    alone.forces()
    alone.step(steps, graph=True)
    alone.forces()
    ms1g = _timed(alone.stream, lambda: alone.step(steps, graph=True)) / steps
    alone.forces()
    alone.close()
    out["one_slab_ms_per_step"] = round(ms1, 4)
    out["one_slab_graph_ms_per_step"] = round(ms1g, 4)
    best1 = min(ms1, ms1g)
    out["one_slab_MLUPS"] = round(w * prob.ny / (best1 * 1e-3) / 1e6, 1)
    out["projected_n_gpu_MLUPS"] = round(n_slabs * w * prob.ny / (best1 * 1e-3) / 1e6, 1)
    # weak scaling: every GPU holds a slab as large as the whole domain here, closed
    # on itself through its own exchange (its two cuts' transfers)
    big = inputs.split_x(dataclasses.replace(prob, bc=("periodic", "periodic", "periodic", "periodic")),
                         [prob.nx])[0]
    full = lbvp.Slabs(big, [0], storage=storage, force_every=1, force_capacity=steps + 16)
    full.step(5)
    full.forces()
    full.step(steps, graph=True)
    full.forces()
    msw = _timed(full.stream, lambda: full.step(steps, graph=True)) / steps
    full.forces()
    full.close()
    torch.cuda.empty_cache()
    out["weak_slab"] = f"{prob.nx}x{prob.ny} per GPU"
    out["weak_slab_ms_per_step"] = round(msw, 4)
    out["projected_n_gpu_weak_MLUPS"] = round(n_slabs * nodes / (msw * 1e-3) / 1e6, 1)
    return out


def _host_cpu():
    """CPU model name and processor counts of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def _oracle_rate(ref, prob, budget_s: float, threads: int):
    """Whole FP64 steps of prob on `threads` threads for about budget_s seconds
    (at least one): (MLUPS, steps, seconds)."""
    ref.set_num_threads(threads)
    r = ref.RefSolver(prob)
    t0 = time.perf_counter()
    r.step(1)
    one = time.perf_counter() - t0
    n_more = max(0, int(0.8 * budget_s / max(one, 1e-9)) - 1)
    t1 = time.perf_counter()
    if n_more:
        r.step(n_more)
    total = one + (time.perf_counter() - t1)
    r.close()
    steps = 1 + n_more
    return prob.nx * prob.ny * steps / total / 1e6, steps, total


def cpu_baseline(prob, budget_s: float = 15.0):
    """The FP64 oracle on this host's cores, on the same domain, for as many
    whole steps as fit in about ``budget_s`` seconds (at least one); then one
    step on a single thread for the per-core rate; then the 1024 x 512 cylinder
    (the shedding case) on all threads for about a third of the budget."""
    from oracle import ref
    from paper_1901_08766_amd import inputs

    cores = ref.num_threads()
    mlups, steps, total = _oracle_rate(ref, prob, budget_s, cores)
    single, _, single_s = _oracle_rate(ref, prob, 0.0, 1)
    c2 = inputs.cylinder()
    c2_mlups, c2_steps, c2_s = _oracle_rate(ref, c2, budget_s / 3.0, cores)
    ref.set_num_threads(cores)
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "single_thread_MLUPS": round(single, 3), **_host_cpu(),
            "cylinder_1024x512_MLUPS": round(c2_mlups, 3),
            "sample": f"{steps} FP64 steps of the full {prob.nx}x{prob.ny} domain on {cores} threads "
                      f"({total:.1f} s), then 1 step on 1 thread ({single_s:.1f} s), then {c2_steps} steps of the "
                      f"1024x512 cylinder on {cores} threads ({c2_s:.1f} s)"}


def _timed(stream, fn):
    import torch

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def time_ensemble(storage: str, steps: int, per_domain_steps: int, n_dom: int = 256, graph_chunk: int = 20):
    """The batched ensemble (uneven domains, one launch per step over all of them,
    launch shape and layout from the tuner) against the plain kernel launched per
    domain per step, domains round-robin on one stream, at the same storage
    type; both also through HIP graphs."""
    import torch
    from paper_1901_08766_amd import inputs, lbvp

    probs = inputs.ensemble(n=n_dom)
    nodes = sum(p.nx * p.ny for p in probs)
    stream = torch.cuda.Stream()
    cap = max(steps, per_domain_steps) + 64

    def make(flags):
        return [lbvp.Solver(p, storage=storage, force_every=1, force_capacity=cap, flags=flags, stream=stream)
                for p in probs]

    def drain(ms):
        for m in ms:
            m.forces()

    members = make(0)
    defaults = [m.launch for m in members]
    rows, best = lbvp.tune(members, steps=40, layouts=True)
    out = {"domains": n_dom, "nodes": nodes, "storage": storage,
           "tuned": {"layout": "aa" if best["layout_flags"] else "pull", "vec": best["vec"], "block": best["block"],
                     "tile_band": best["band"]},
           "tuner_rows": len(rows)}
    # per-domain plain launches (pull layout, each domain's default launch shape)
    for m in members:
        m.step(2)
    stream.synchronize()
    drain(members)

    def per_domain():
        for _ in range(per_domain_steps):
            for m in members:
                m.step(1)

    ms = _timed(stream, per_domain)
    out["per_domain_MLUPS"] = round(nodes * per_domain_steps / ms / 1e3, 1)
    drain(members)
    for m in members:
        m.step(graph_chunk, graph=True)       # capture outside the timed region
    stream.synchronize()
    drain(members)

    def per_domain_graph():
        for _ in range(per_domain_steps // graph_chunk):
            for m in members:
                m.step(graph_chunk, graph=True)

    ms = _timed(stream, per_domain_graph)
    out["per_domain_graph_MLUPS"] = round(nodes * (per_domain_steps // graph_chunk) * graph_chunk / ms / 1e3, 1)
    drain(members)
    assert all(m.launch == d for m, d in zip(members, defaults))
    if best["layout_flags"]:
        for m in members:
            m.close()
        members = make(lbvp.LAYOUT_AA)
    batch = lbvp.Batch(members, vec=best["vec"], block=best["block"])
    batch.set_tile_band(best["band"])
    batch.step(10)
    batch.step(steps, graph=True)             # capture outside the timed region
    stream.synchronize()
    drain(members)
    ms = _timed(stream, lambda: batch.step(steps))
    out["batched_MLUPS"] = round(nodes * steps / ms / 1e3, 1)
    out["batched_ms_per_step"] = round(ms / steps, 4)
    drain(members)
    ms = _timed(stream, lambda: batch.step(steps, graph=True))
    out["batched_graph_MLUPS"] = round(nodes * steps / ms / 1e3, 1)
    _, mass, _ = members[0].forces()
    out["finite"] = bool(np.isfinite(mass).all())
    drain(members)
    out["steps"] = {"batched": steps, "per_domain": per_domain_steps}
    out["batched_vs_per_domain"] = round(out["batched_MLUPS"] / out["per_domain_MLUPS"], 2)
    launch = {"vec": best["vec"], "block": best["block"]}
    bpn = sum(alg_bytes_per_node(storage, p, launch) * p.nx * p.ny for p in probs) / nodes
    out["alg_bytes_per_node"] = round(bpn, 3)
    out["hbm_frac_batched"] = round(out["batched_MLUPS"] * 1e6 * bpn / (HBM_PEAK_GBPS * 1e9), 4)
    batch.close()
    for m in members:
        m.close()
    torch.cuda.empty_cache()
    return out


def profile_ensemble(storage: str, launch, steps: int, warmup: int):
    """Only the batched 256-domain ensemble in one given launch shape (vec, block,
    band): warmup steps, then `steps` timed ones (for kernel traces and counters,
    without the tuner's and the per-domain runs' launches)."""
    import torch
    from paper_1901_08766_amd import inputs, lbvp

    probs = inputs.ensemble(n=256)
    nodes = sum(p.nx * p.ny for p in probs)
    stream = torch.cuda.Stream()
    members = [lbvp.Solver(p, storage=storage, force_every=1, force_capacity=steps + warmup + 16, stream=stream)
               for p in probs]
    vec, block, band = launch
    batch = lbvp.Batch(members, vec=vec, block=block)
    batch.set_tile_band(band)
    batch.step(warmup)
    stream.synchronize()
    for m in members:
        m.forces()
    ms = _timed(stream, lambda: batch.step(steps))
    bpn = sum(alg_bytes_per_node(storage, p, {"vec": vec, "block": block}) * p.nx * p.ny for p in probs) / nodes
    out = {"ensemble_profile": storage, "launch": list(launch), "nodes": nodes, "steps": steps,
           "ms_per_step": round(ms / steps, 4), "MLUPS": round(nodes * steps / ms / 1e3, 1),
           "alg_bytes_per_node": round(bpn, 3),
           "hbm_frac": round(nodes * steps / ms * 1e3 * bpn / (HBM_PEAK_GBPS * 1e9), 4),
           "traffic": measured_traffic(storage, nodes, key="ensemble_" + storage)}
    batch.close()
    for m in members:
        m.close()
    return out


def run_serving(storage: str, rate: float, n_req: int, seed: int = 5, max_slots: int = 256,
                max_epoch_steps: int = 256, tune_sample: int = 32):
    """Poisson arrivals of cylinder and airfoil solves through the native pool;
    p50/p99 latency and aggregate MLUPS over the whole run (first arrival to
    last result on the host)."""
    import torch
    from paper_1901_08766_amd import inputs, lbvp, serve

    reqs = inputs.request_stream(rate=rate, n=n_req, seed=seed)
    best = serve.sample_pool_shape([r.problem for r in reqs[:tune_sample]], storage)
    pool = lbvp.Pool(storage=storage, layout_aa=bool(best["layout_flags"]), cap_bytes=200 * 10**9,
                     max_slots=max_slots, vec=best["vec"], block=best["block"])
    finite = []
    rep = serve.serve(reqs, pool, max_epoch_steps=max_epoch_steps,
                      on_result=lambda r, f, m, _: finite.append(bool(np.isfinite(m).all())))
    st = pool.stats()
    pool.close()
    torch.cuda.empty_cache()
    out = {"storage": storage, "rate_req_per_s": rate, **rep.summary(),
           "pool": {"layout": "aa" if best["layout_flags"] else "pull", "vec": best["vec"], "block": best["block"],
                    "max_slots": max_slots, "cap_bytes": 200 * 10**9, "max_epoch_steps": max_epoch_steps,
                    "reserved_bytes": st["reserved_bytes"]},
           "mean_steps": round(float(np.mean([r.problem.steps for r in reqs])), 1),
           "all_finite": all(finite)}
    return out


def _rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / max(np.sum(b ** 2), 1e-300)))


def precision_study(checkpoints=(1000, 5000, 50000), rec_every: int = 10):
    """Reduced-storage error of the large 8192 x 4096 domain against an FP64 run on
    the GPU (whose arithmetic matches the oracle to 1e-12): per-field rel-L2 of
    (rho - 1, u_x, u_y) at the checkpoints, and per-body C_d mean / C_l amplitude
    over the second half of the run."""
    from paper_1901_08766_amd import diagnostics, inputs, lbvp

    prob = inputs.large_domain()
    last = checkpoints[-1]
    cap = last // rec_every + 16
    runs = {st: lbvp.Solver(prob, storage=st, force_every=rec_every, force_capacity=cap)
            for st in ("f64", "f32", "f16", "bf16")}
    forces = {st: [] for st in runs}
    out = {"workload": f"{prob.name}, Re 200, U 0.04", "checkpoints": {}}
    done = 0
    for cp in checkpoints:
        fl = {}
        for st, s in runs.items():
            s.step(cp - done, keep_fields=True)
            try:
                f, _, _ = s.forces()
            except lbvp.LbvpError as e:
                f, _, _ = e.data
            forces[st].append(f)
            fl[st] = s.fields()
        done = cp
        ref = fl["f64"]
        row = {}
        for st in ("f32", "f16", "bf16"):
            row[st] = {"rho": _rel_l2(fl[st]["rho"] - 1.0, ref["rho"] - 1.0), "ux": _rel_l2(fl[st]["ux"], ref["ux"]),
                       "uy": _rel_l2(fl[st]["uy"], ref["uy"])}
        out["checkpoints"][str(cp)] = row
        print(f"# precision at step {cp}: {row}", file=sys.stderr, flush=True)
        del fl
    half = last // rec_every // 2
    stats = {}
    for st in runs:
        f = np.concatenate(forces[st])[half:]
        # a 50k-step run holds about one shedding period at D = 160, so no Strouhal number
        stats[st] = [{k: v for k, v in diagnostics.shedding(f[:, b], rec_every, prob.u_ref,
                                                             prob.l_ref if b < 4 else 5 * prob.l_ref).items()
                      if k != "st"} for b in range(prob.n_bodies)]
    out["body_stats_second_half"] = stats
    for s in runs.values():
        s.close()
    return out


def steady_wake(res=(20.0, 40.0), steps: int = 60000, storages=("f32", "f64")):
    """The single cylinder (1024 x 512, D = 40, U = 0.05) at low Re run to a steady
    state: C_d from the force record, recirculation length L_s/D and separation
    angle theta_s from the final fields."""
    from paper_1901_08766_amd import diagnostics, inputs, lbvp

    out = []
    for re in res:
        for st in storages:
            prob = inputs.cylinder(re=re, noise=False)
            s = lbvp.Solver(prob, storage=st, force_every=100, force_capacity=steps // 100 + 8)
            s.step(steps - 1000)
            s.forces()
            s.step(1000, keep_fields=True)
            f, _, _ = s.forces()
            fields = s.fields()
            cd, cl = diagnostics.force_coefficients(f[-1, 0], prob.u_ref, prob.l_ref)
            drift = float(abs(diagnostics.force_coefficients(f[0, 0], prob.u_ref, prob.l_ref)[0] - cd) / abs(cd))
            cx, cy = prob.bodies[0, 0], prob.bodies[0, 1]
            ls, th = diagnostics.steady_wake(fields, cx, cy, prob.l_ref / 2.0)
            row = {"re": re, "storage": st, "steps": steps, "cd": round(float(cd), 5), "cl": round(float(cl), 6),
                   "cd_drift_last_1000_steps": drift, "ls_over_d": round(ls, 4), "theta_s_deg": round(th, 2)}
            print(json.dumps(row), flush=True)
            out.append(row)
            s.close()
    return out


def copy_bandwidth(nbytes: int = 2415919104, reps: int = 20) -> float:
    """GB/s (bytes read + written) of the library's device copy (one 16-byte
    non-temporal load and store per thread, the fastest copy form measured) over
    nbytes each way, about what one 8192x4096 FP32 step moves."""
    import torch
    from paper_1901_08766_amd import lbvp

    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    s = torch.cuda.Stream()
    lbvp.lbvp_device_copy(a.data_ptr(), b.data_ptr(), nbytes, s.cuda_stream)
    ms = _timed(s, lambda: [lbvp.lbvp_device_copy(a.data_ptr(), b.data_ptr(), nbytes, s.cuda_stream)
                            for _ in range(reps)]) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / ms / 1e6


def calibrate_copy(nbytes: int, reps: int = 5):
    """A plain device copy of known size (torch's copy kernel): what the HBM
    traffic counters read for it calibrates them, and its rate is the copy
    bandwidth this device reaches."""
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"calibration": "device copy", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                      "copies": reps + 1, "ms_per_copy": round(ms, 4),
                      "GBps": round(2 * nbytes / ms / 1e6, 1)}), flush=True)


def _db_rows(db: str, table: str):
    import sqlite3

    con = sqlite3.connect(db)
    cols = [d[1] for d in con.execute(f"pragma table_info({table})")]
    return [dict(zip(cols, r)) for r in con.execute(f"select * from {table}")]


def summarize_trace(db: str, out: str, command: str):
    """Write the per-kernel statistics of a rocprofv3 --kernel-trace --stats run."""
    rows = _db_rows(db, "top_kernels")
    lines = ["# rocprofv3 kernel-trace summary", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | average (us) | total (us) | share |", "|---|---|---|---|---|"]
    for r in rows[:12]:
        lines.append(f"| `{r['name'][:100]}` | {r['total_calls']} | {r['average']:.2f} | "
                     f"{r['total_duration']:.1f} | {r['percentage']:.1f}% |")
    if rows:   # per-dispatch spread and resources of the dominant kernel
        top = rows[0]["name"]
        ks = [k for k in _db_rows(db, "kernels") if k["name"] == top]
        d = sorted(k["duration"] / 1e3 for k in ks)
        k0 = ks[0]
        lines += ["", f"Dominant kernel: {len(d)} dispatches, duration median {d[len(d) // 2]:.2f} us, "
                      f"min {d[0]:.2f} us, max {d[-1]:.2f} us; {k0['grid_x']} work-items in {k0['workgroup_x']}-thread "
                      f"workgroups, {k0['vgpr_count']} VGPRs, {k0['accum_vgpr_count']} AGPRs, "
                      f"{k0['sgpr_count']} SGPRs, {k0['lds_size']} B LDS, {k0['scratch_size']} B scratch."]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter_mean(db: str, counter: str, name_part: str) -> float:
    vals = [r["value"] for r in _db_rows(db, "counters_collection")
            if r["counter_name"] == counter and name_part in (r["kernel_name"] or "")]
    if not vals:
        raise SystemExit(f"no {counter} values for kernels matching {name_part!r} in {db}")
    return sum(vals) / len(vals)


def summarize_counters(step_fetch: str, step_write: str, copy_fetch: str, copy_write: str, copy_bytes: int,
                       storage: str, kernel_part: str, out_md: str, command: str, lattice: str = "d2q9",
                       ensemble_launch=None):
    """HBM bytes per step-kernel launch from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled by what the counter reads for a plain device copy of
    copy_bytes read and copy_bytes written. ensemble_launch: the counters are of
    the batched 256-domain ensemble in that launch shape (entry ensemble_<storage>)."""
    key = storage
    if lattice == "d2q9" and ensemble_launch is not None:
        from paper_1901_08766_amd import inputs
        probs = inputs.ensemble(n=256)
        nodes = sum(p.nx * p.ny for p in probs)
        mask_bytes = int(round(sum(mask_read_fraction(p, ensemble_launch) * p.nx * p.ny for p in probs)))
        key = "ensemble_" + storage
    elif lattice == "d2q9":
        from paper_1901_08766_amd import inputs
        prob = inputs.large_domain()
        nodes = prob.nx * prob.ny
        # the mask bytes of the tiles holding a solid node, in the default launch
        # that the profiled command runs
        mask_bytes = int(round(mask_read_fraction(prob, DEFAULT_LAUNCH_2D[storage]) * nodes))
    else:
        from paper_1901_08766_amd import inputs3
        prob = inputs3.sphere()
        nodes = int(np.prod(inputs3.SPHERE_SHAPE))
        mask_bytes = int(round(mask_read_fraction(prob, DEFAULT_LAUNCH_3D[storage]) * nodes))
    out_json = LATTICES[lattice]["counters"]
    pop_bytes = LATTICES[lattice]["q"] * STORAGE_BYTES[storage]
    copy_kib = copy_bytes / 1024.0
    f_cal = copy_kib / _counter_mean(copy_fetch, "FETCH_SIZE", "copyBuffer")
    w_cal = copy_kib / _counter_mean(copy_write, "WRITE_SIZE", "copyBuffer")
    fk = _counter_mean(step_fetch, "FETCH_SIZE", kernel_part)
    wk = _counter_mean(step_write, "WRITE_SIZE", kernel_part)
    fetch_b = fk * f_cal * 1024.0
    write_b = wk * w_cal * 1024.0
    alg_read = pop_bytes * nodes + mask_bytes   # every population once, the mask where it is read
    alg_write = pop_bytes * nodes
    entry = {"nodes": nodes, "fetch_kib_raw": round(fk, 1), "write_kib_raw": round(wk, 1),
             "fetch_calibration": round(f_cal, 5), "write_calibration": round(w_cal, 5),
             "hbm_fetch_bytes": int(fetch_b), "hbm_write_bytes": int(write_b),
             "hbm_bytes_per_launch": int(fetch_b + write_b),
             "algorithmic_read_bytes": alg_read, "algorithmic_write_bytes": alg_write,
             "fetch_over_algorithmic": round(fetch_b / alg_read, 4),
             "write_over_algorithmic": round(write_b / alg_write, 4)}
    entry["kernel"] = kernel_part
    entry["command"] = command
    # one entry per storage type, kept while they describe the same kernel source
    try:
        with open(out_json) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    if data.get("kernel_source_hash") != kernel_source_hash(lattice):
        data = {"kernel_source_hash": kernel_source_hash(lattice), "per_storage": {}}
    data.pop("kernel", None)
    data.pop("command", None)
    data.setdefault("per_storage", {})[key] = entry
    with open(out_json, "w") as f:
        json.dump(data, f, indent=1)
    md = ["# HBM traffic of the step kernel (rocprofv3 PMC)", "", "Command:", "", "```", command, "```", "",
          f"Kernel `{kernel_part}`, {nodes} nodes, storage {storage}, kernel source hash "
          f"`{data['kernel_source_hash']}`.", "",
          "| quantity | value |", "|---|---|"]
    for k, v in entry.items():
        md.append(f"| {k} | {v} |")
    md += ["", f"Calibration: a device copy of {copy_bytes} bytes read and written reads "
               f"FETCH_SIZE x {f_cal:.4f} and WRITE_SIZE x {w_cal:.4f} of its true bytes; the step "
               f"kernel's counters are scaled by these factors."]
    with open(out_md, "w") as f:
        f.write("\n".join(md) + "\n")
    print("\n".join(md))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=sorted(POP_BYTES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--variants", default="f16,bf16,f64",
                    help="other storage types to time as extra fields ('' for none)")
    ap.add_argument("--moving-storages", default="f32,f16",
                    help="storage types to time on the large domain with moving masks ('' for none)")
    ap.add_argument("--ensemble-steps", type=int, default=300,
                    help="batched steps of the 256-domain ensemble comparison (0: skip it)")
    ap.add_argument("--ensemble-storages", default="f32,f16")
    ap.add_argument("--d3q19-steps", type=int, default=50,
                    help="timed steps of the D3Q19 sphere domain (0: skip it)")
    ap.add_argument("--d3q19-storages", default="f32,f16,f64")
    ap.add_argument("--d3q19-ensemble-steps", type=int, default=None,
                    help="timed steps of the D3Q19 ensemble, batched and per domain (0: skip it; "
                         "default 100, and none with --d3q19-only)")
    ap.add_argument("--d3q19-ensemble-storages", default="f32,f16")
    ap.add_argument("--d3q19-only", action="store_true", help="only run the D3Q19 timing leg")
    ap.add_argument("--slabs", type=int, default=0, metavar="N",
                    help="only time the large domain as N x-slabs on this GPU (halo exchange + batched step)")
    ap.add_argument("--lattice", default="d2q9", choices=sorted(LATTICES),
                    help="the step kernel --summarize-counters describes")
    ap.add_argument("--serve-requests", type=int, default=100,
                    help="requests of the serving sample (0: skip it)")
    ap.add_argument("--serve-rate", type=float, default=100.0)
    ap.add_argument("--serve-storage", default="f16")
    ap.add_argument("--serve-sweep", default="",
                    help="only run the serving stream at these comma-separated rates (req/s)")
    ap.add_argument("--ensemble-profile", default="", metavar="STORAGE",
                    help="only run the batched 256-domain ensemble in --ensemble-launch for --steps steps")
    ap.add_argument("--ensemble-launch", default="8,64,16", help="vec,block,band of --ensemble-profile")
    ap.add_argument("--counters-ensemble", action="store_true",
                    help="--summarize-counters describes the ensemble profile in --ensemble-launch")
    ap.add_argument("--precision-study", action="store_true",
                    help="only run FP32/FP16/BF16 against FP64 on the large domain (1k/5k/50k steps)")
    ap.add_argument("--steady-wake", action="store_true",
                    help="only run the low-Re steady cylinder diagnostics (Re 20 and 40)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("DB", "OUT_MD", "COMMAND"),
                    help="write the kernel statistics of a rocprofv3 kernel-trace database")
    ap.add_argument("--summarize-counters", nargs=8,
                    metavar=("STEP_FETCH_DB", "STEP_WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB", "COPY_BYTES",
                             "KERNEL", "OUT_MD", "COMMAND"),
                    help="write the calibrated HBM traffic of the step kernel from four rocprofv3 PMC runs")
    a = ap.parse_args()
    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return
    if a.summarize_trace:
        summarize_trace(*a.summarize_trace)
        return
    ens_launch = tuple(int(x) for x in a.ensemble_launch.split(","))
    if a.summarize_counters:
        sf, sw, cf, cw, cb, kern, md, cmd = a.summarize_counters
        summarize_counters(sf, sw, cf, cw, int(cb), a.storage, kern, md, cmd, a.lattice,
                           {"vec": ens_launch[0], "block": ens_launch[1]} if a.counters_ensemble else None)
        return
    if a.ensemble_profile:
        print(json.dumps(profile_ensemble(a.ensemble_profile, ens_launch, a.steps, a.warmup)), flush=True)
        return
    if a.slabs:
        print(json.dumps(time_slabs(a.slabs, storage=a.storage)), flush=True)
        return
    if a.d3q19_only:
        res = time_d3q19([x for x in a.d3q19_storages.split(",") if x], a.d3q19_steps, a.warmup) \
            if a.d3q19_steps > 0 else {}
        if a.d3q19_ensemble_steps:
            res["ensemble"] = {st: time_ensemble3(st, a.d3q19_ensemble_steps)
                               for st in a.d3q19_ensemble_storages.split(",") if st}
        print(json.dumps(res), flush=True)
        return
    if a.precision_study:
        print(json.dumps(precision_study()), flush=True)
        return
    if a.steady_wake:
        steady_wake()
        return
    if a.serve_sweep:
        for rate in [float(x) for x in a.serve_sweep.split(",")]:
            print(json.dumps(run_serving(a.serve_storage, rate, a.serve_requests)), flush=True)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the single-domain step has "
                                   "no multi-GPU path in this build (--gpus must be 1)"}))
        sys.exit(2)

    from paper_1901_08766_amd import inputs

    prob = inputs.large_domain()
    nodes = prob.nx * prob.ny
    print(f"# workload {prob.name}: {nodes} nodes, {prob.n_bodies} bodies, storage {a.storage}", file=sys.stderr,
          flush=True)
    # the plain device copy (the practical bandwidth ceiling the step is compared
    # with) is measured first
    copy_gbps = copy_bandwidth()
    ms, ok, launch = time_gpu(a.storage, a.steps, a.warmup, prob)
    if not ok:
        raise SystemExit("non-finite mass during the timed run")
    mlups = nodes / (ms * 1e-3) / 1e6
    bpn = alg_bytes_per_node(a.storage, prob, launch)
    alg_bytes = bpn * nodes
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    extra, moving_res = {}, {}
    for v in [s for s in a.variants.split(",") if s and s != a.storage]:
        # median of 5 repeats of the requested steps (the first absorbs the
        # clock ramp after the set-up of the variant's context)
        vms, vok, vlaunch, vruns = time_gpu(v, a.steps, a.warmup, prob, repeats=5)
        vbpn = alg_bytes_per_node(v, prob, vlaunch)
        vb = vbpn * nodes / (vms * 1e-3) / 1e9
        extra[v] = {"alg_bytes_per_node": round(vbpn, 3), "MLUPS": round(nodes / (vms * 1e-3) / 1e6, 1), "ms_per_step": round(vms, 4),
                    "ms_per_step_runs": [round(x, 4) for x in vruns],
                    "timing": f"median of 5 repeats of {a.steps} steps after {a.warmup} + 100 untimed steps",
                    "achieved_GBps": round(vb, 1), "hbm_frac": round(vb / HBM_PEAK_GBPS, 4), "finite": vok,
                    "launch": vlaunch, "traffic": measured_traffic(v, nodes)}
        print(f"# {v}: {extra[v]}", file=sys.stderr, flush=True)
    if a.moving_storages:
        # the same domain with its masks following the bodies (a cylinder crossing
        # the stream, the airfoil pitching, the rotating pair turning their masks)
        mprob = inputs.large_domain(moving=True)
        for v in [s for s in a.moving_storages.split(",") if s]:
            vms, vok, vlaunch, vruns = time_gpu(v, a.steps, a.warmup, mprob, repeats=5)
            vbpn = alg_bytes_per_node(v, mprob, vlaunch)
            vb = vbpn * nodes / (vms * 1e-3) / 1e9
            fixed = ms if v == a.storage else extra.get(v, {}).get("ms_per_step")
            moving_res[v] = {"alg_bytes_per_node": round(vbpn, 3), "MLUPS": round(nodes / (vms * 1e-3) / 1e6, 1), "ms_per_step": round(vms, 4),
                             "ms_per_step_runs": [round(x, 4) for x in vruns], "finite": vok, "launch": vlaunch,
                             "achieved_GBps": round(vb, 1), "hbm_frac": round(vb / HBM_PEAK_GBPS, 4),
                             "time_vs_fixed_mask": round(vms / fixed, 4) if fixed else None}
            print(f"# moving {v}: {moving_res[v]}", file=sys.stderr, flush=True)
    traffic = measured_traffic(a.storage, nodes)
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.storage,
        "data": "synthetic",
        "config": {"workload": f"large single domain {prob.nx}x{prob.ny}, 5 bodies (counter-rotating pair, "
                               f"tandem pair, NACA-0012), Re=200, U=0.04",
                   "nx": prob.nx, "ny": prob.ny, "storage": a.storage, "layout": "two-lattice pull",
                   "force_every": 1},
        "launch": launch,
        "alg_bytes_per_node": round(bpn, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic},
        "variants": extra,
        "moving_bodies": {"workload": f"the same {prob.nx}x{prob.ny} domain with time-dependent masks: the "
                                      "upstream tandem cylinder crossing at 0.1 U, the airfoil pitching "
                                      "(trailing edge 0.3 U), the rotating pair turning their masks",
                          "timing": f"median of 5 repeats of {a.steps} steps, default launch",
                          **moving_res} if moving_res else None,
        "copy": {"GBps": round(copy_gbps, 1), "step_frac_of_copy": round(achieved / copy_gbps, 4),
                 "kernel": "device copy, one 16-byte non-temporal load and store per thread (lbvp_device_copy), 2.4 GB each way"},
    }
    if a.ensemble_steps > 0:
        out["ensemble"] = {}
        for st in [x for x in a.ensemble_storages.split(",") if x]:
            out["ensemble"][st] = time_ensemble(st, a.ensemble_steps, max(20, a.ensemble_steps // 5))
            print(f"# ensemble {st}: {out['ensemble'][st]}", file=sys.stderr, flush=True)
    if a.d3q19_steps > 0:
        out["d3q19"] = time_d3q19([x for x in a.d3q19_storages.split(",") if x], a.d3q19_steps, a.warmup)
    if a.d3q19_ensemble_steps is None:
        a.d3q19_ensemble_steps = 100
    if a.d3q19_ensemble_steps > 0:
        out.setdefault("d3q19", {})["ensemble"] = {
            st: time_ensemble3(st, a.d3q19_ensemble_steps) for st in a.d3q19_ensemble_storages.split(",") if st}
    if a.serve_requests > 0:
        out["serving"] = run_serving(a.serve_storage, a.serve_rate, a.serve_requests)
        print(f"# serving: {out['serving']}", file=sys.stderr, flush=True)
        # a sub-capacity point and one more loaded point, fewer requests each
        out["serving_sweep"] = []
        for rate in (20.0, 200.0):
            row = run_serving(a.serve_storage, rate, max(10, a.serve_requests // 2))
            out["serving_sweep"].append(row)
            print(f"# serving {rate:g} req/s: {row}", file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, a.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
