#!/usr/bin/env python3
"""RTG-GMRES throughput on one MI355X: solves/s at 512x512x3, m = 50.

A step is one call of the batched solver over a batch of B independent
512x512x3 colour deblurring problems (the paper's Example-1 setting at the
sizes of the headline workload: Gaussian blur sigma 2.5 with half-bandwidth
8, 3x3 channel mix, noise 1e-3, sketch 64x64x3, discrepancy-principle mu).
Inputs are synthetic and resident in HBM before the timed region.

Variants (each timed over the same number of steps):
  fp32_plain     float32 basis and MFMA, X0 = 0, m = 50 (the plain solver)
  bf16_warm      bfloat16 basis and MFMA, started from a warm start X0;
                 --x0 learned uses the trained warm-start network (if its
                 weights exist), --x0 observation uses X0 = C.  Stops at the
                 discrepancy level (at most --m-warm steps); the plain float32
                 solver (X0 = 0, m = 50) re-solves, inside the timed step, any
                 problem that does not get there (rtg_solve_batched_fallback)
  bf16_obs       bf16_warm from X0 = C instead of the network's X0: the same
                 stop rule, step limit and fallback, so the pair shows the
                 steps and solves/s the trained network buys
  fp32_unsketched  fp32_plain with the identity sketch (Frobenius inner
                 products: the unsketched global GMRES)
  fp32_gk        sketched Block Golub-Kahan (Sec. 4.5), float32 basis,
                 X0 = 0, m = 50 columns
  fp32_psf       the same images blurred by a 9x9 non-separable PSF
                 (rotated anisotropic Gaussian, eq. (57)), float32 basis,
                 m = 50 (W sketched after it is formed)
  fp32_uneven    256 images of uneven size (sides 64..512, sigma U(1,3),
                 noise U[1e-3, 1e-2], sketches of a quarter of each mode) in
                 one batch, float32 basis, X0 = 0, m = 40; solves/s counts
                 those 256 problems per step.  (A bfloat16 basis from X0 = 0
                 misses the oracle's restoration error on this batch: some
                 problems do not reach the discrepancy level in 40 steps.)
  mixed_uneven   the same batch in the mixed form RTG_F32_BF16: float32 basis,
                 sketch contractions on bfloat16 MFMA operands with float32
                 accumulation
  mixed_uneven_persist  mixed_uneven with its Arnoldi process in one
                 persistent launch (rtg_tune.persist = 1; the other shapes
                 autotuned)
  fp32_video     --video-batch 256x256x64 grayscale videos (spatial sigma 2,
                 temporal box blur of width 5, noise 1e-3, sketch 48x48x16),
                 float32 basis, X0 = 0, m = 80
  bf16_video     the same videos, bfloat16 basis from X0 = C, m = 80
Each batch is autotuned (rtg_autotune_batched) before its timed region
unless --no-autotune; the chosen launch shapes are reported.
The JSON line reports the headline variant in "value" and every variant
under "variants", with restoration errors (RE) against the ground truth, the
count of each flag value over the batch, the fallback re-solves per step,
and the ratio of RE to the float64 oracle's RE on sampled problems: the
oracle solves problems 0 and 1 of the 512x512x3 batch and problem 0 of the
non-separable PSF batch in the CPU-baseline leg; the uneven-batch and video
figures are the stored oracle results of tests/golden/oracle_re.json (the
oracle takes minutes there).  The oracle forms its own observation C from
the same seeded inputs (the GPU forms C with its operator: the two differ by
float32 rounding only).

Live measurement: the dominant byte mover of the headline variant (the
fused Arnoldi step kernel for the bfloat16 basis, the multi-AXPY tile kernel
for the float32 one) is bracketed by HIP events on its launch stream inside
the library; its algorithmic bytes (the tensor reads and writes the method
needs) over its measured time give the roofline entry.  "traffic" is the
rocprofv3-measured HBM traffic per launch recorded under profiles/ for the
same kernel source and launch shapes (null once either differs).  The CPU baseline
times the float64 oracle on problems of the same workload on the host
cores, with every BLAS thread and with one, and records the core count and
the CPU model.

--copy-calibration MB runs only a device-to-device copy of MB megabytes
(three times), the plain copy kernel that calibrates the rocprofv3
FETCH_SIZE / WRITE_SIZE counters.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RTG-GMRES solves/s at 512²×3, m=50: plain FP32 vs BF16+learned X₀ at equal rel err"
HBM_PEAK_GBS = 8000.0
VARIANTS = ["fp32_plain", "bf16_warm", "bf16_obs", "fp32_unsketched", "fp32_gk", "fp32_psf", "fp32_uneven",
            "mixed_uneven", "mixed_uneven_persist", "fp32_video", "bf16_video"]
# the plain solver that re-solves failed warm starts: X0 = 0, m = 50, float32 basis
FALLBACK_M = 50
GOLDEN_RE = os.path.join(ROOT, "tests", "golden", "oracle_re.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--m", type=int, default=50)
    ap.add_argument("--m-warm", type=int, default=10, help="Arnoldi steps of the warm-started BF16 solve")
    ap.add_argument("--warm-stop", choices=["fixed", "discrepancy"], default="discrepancy",
                    help="warm-started solve: run --m-warm steps, or stop at the first step whose projected "
                         "least-squares residual is within the discrepancy level eta*delta (at most --m-warm)")
    ap.add_argument("--x0", choices=["learned", "observation"], default="learned")
    ap.add_argument("--overlap", choices=["on", "off"], default="on",
                    help="bf16_warm: run the next batch's network while the host waits for the fallback flags")
    ap.add_argument("--headline", choices=["auto", "fp32_plain", "bf16_warm"], default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--video-batch", type=int, default=4, help="videos per step of the video variants")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time every batch with the library's default launch shapes")
    ap.add_argument("--tune", default="", metavar="FIELD=V,...",
                    help="time every batch with these launch shapes (rtg_tune fields; the rest default), "
                         "no autotuning")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a device-to-device copy of MB megabytes (counter calibration)")
    ap.add_argument("--only", choices=VARIANTS,
                    default=None,
                    help="time one variant only (profiling runs)")
    return ap.parse_args()


def make_batch(B, device):
    """B cfg2 problems (seeds 0..B-1): ground truth, observation C formed on
    the GPU with the library's operator plus scaled Gaussian noise."""
    import numpy as np
    import torch
    from paper_2603_00839_amd import rtg, synth
    probs = []
    op = None
    for b in range(B):
        p = synth.cfg2(b)
        if op is None:
            op = rtg.setup_operator(*p.dims, p.a1_band, p.a2_band, p.b_band)
        sk = rtg.setup_sketch(*p.dims, p.om1, p.om2, p.om3)
        xt = torch.from_numpy(synth.to_device_layout(p.x_true)).to(device)
        g = torch.from_numpy(synth.to_device_layout(p.noise_dir)).to(device)
        chat = rtg.apply_operator(op, xt)
        delta = p.nu * float(torch.linalg.vector_norm(chat.double()))
        C = (chat + g * (delta / float(torch.linalg.vector_norm(g.double())))).contiguous()
        probs.append(dict(p=p, sk=sk, xt=xt, C=C, delta=delta))
    return op, probs


def make_psf_batch(B, device):
    """B problems of the non-separable PSF workload (seeds 0..B-1), the
    observation formed on the GPU with the library's operator plus noise."""
    import torch
    from paper_2603_00839_amd import rtg, synth
    probs = []
    op = None
    for b in range(B):
        p = synth.cfg2_psf(b)
        if op is None:
            op = rtg.setup_operator_psf(*p.dims, p.psf, p.b_band)
        sk = rtg.setup_sketch(*p.dims, p.om1, p.om2, p.om3)
        xt = torch.from_numpy(synth.to_device_layout(p.x_true)).to(device)
        g = torch.from_numpy(synth.to_device_layout(p.noise_dir)).to(device)
        chat = rtg.apply_operator(op, xt)
        delta = p.nu * float(torch.linalg.vector_norm(chat.double()))
        C = (chat + g * (delta / float(torch.linalg.vector_norm(g.double())))).contiguous()
        probs.append(dict(p=p, sk=sk, xt=xt, C=C, delta=delta))
    return op, probs


def make_video_batch(B, device):
    """B videos of the video workload (256x256x64 grayscale, spatial sigma 2,
    temporal box blur of width 5, noise 1e-3, sketch 48x48x16; seeds
    0..B-1), observations formed on the GPU with the library's operator."""
    import torch
    from paper_2603_00839_amd import rtg, synth
    probs = []
    op = None
    for b in range(B):
        p = synth.cfg3(b)
        if op is None:
            op = rtg.setup_operator(*p.dims, p.a1_band, p.a2_band, p.b_band)
        sk = rtg.setup_sketch(*p.dims, p.om1, p.om2, p.om3)
        xt = torch.from_numpy(synth.to_device_layout(p.x_true)).to(device)
        g = torch.from_numpy(synth.to_device_layout(p.noise_dir)).to(device)
        chat = rtg.apply_operator(op, xt)
        delta = p.nu * float(torch.linalg.vector_norm(chat.double()))
        C = (chat + g * (delta / float(torch.linalg.vector_norm(g.double())))).contiguous()
        probs.append(dict(p=p, sk=sk, xt=xt, C=C, delta=delta))
    return op, probs


def make_uneven_batch(device):
    """The 256 uneven problems (seed 0), observations formed on the GPU with
    each problem's operator plus noise of its level."""
    import numpy as np
    import torch
    from paper_2603_00839_amd import rtg, synth
    probs = []
    for p in synth.cfg4(0, 256, m=40):
        op = rtg.setup_operator(*p.dims, p.a1_band, p.a2_band, p.b_band)
        sk = rtg.setup_sketch(*p.dims, p.om1, p.om2, p.om3)
        xt = torch.from_numpy(synth.to_device_layout(p.x_true)).to(device)
        g = torch.from_numpy(synth.to_device_layout(p.noise_dir)).to(device)
        chat = rtg.apply_operator(op, xt)
        delta = p.nu * float(torch.linalg.vector_norm(chat.double()))
        C = (chat + g * (delta / float(torch.linalg.vector_norm(g.double())))).contiguous()
        probs.append(dict(p=p, op=op, sk=sk, xt=xt, C=C, delta=delta, n=int(np.prod(p.dims))))
    return probs


def rel_err(x, xt):
    import torch
    return float(torch.linalg.vector_norm((x - xt).double()) / torch.linalg.vector_norm(xt.double()))


def step_bytes(n, es, m_eff):
    """Algorithmic HBM bytes of the fused step launches of one bfloat16-basis
    solve: step j reads V_1..V_j and writes V_{j+1}, (j + 1) tensors (the
    operator's re-read of the V_j tile and its halo is not counted again; W is
    never stored).  Steps j = 1 .. m_eff - 1 form a new tensor."""
    return sum((j + 1) * es * n for j in range(1, m_eff))


def frob_bytes(n, es, m_eff):
    """Algorithmic bytes of the Frobenius Gram launches of one unsketched
    solve: step j reads W (float32) and V_1..V_j."""
    return sum(4 * n + j * es * n for j in range(1, m_eff + 1)) + 4 * n


def tile_bytes(n, es, m_eff, has_x0):
    """Algorithmic HBM bytes of the multi-AXPY + sketch tile launches of one
    float32-basis solve: sketch of R0 (reads it), V1 = R0/beta (reads R0,
    writes V1), steps j = 1 .. m_eff - 1 (read V_1..V_j, write V_{j+1}; the
    read of the stored W is not counted: the method does not need W in
    memory), and the assembly X = X0 + V y (reads X0, V_1..V_m, writes X)."""
    b = 2 * 4 * n + es * n
    for j in range(1, m_eff):
        b += (j + 1) * es * n
    b += (4 * n if has_x0 else 0) + m_eff * es * n + 4 * n
    return b


def arnoldi_bytes(n, es, m_eff):
    """Algorithmic HBM bytes of the persistent launch of one float32-basis
    solve (the Arnoldi process without the assembly): the sketch of R0 and
    V1 = R0/beta (read R0 twice, write V1), then steps j = 1 .. m_eff - 1
    (read V_1..V_j, write V_{j+1}).  The operator's W is not counted: the
    method does not need it in memory."""
    b = 2 * 4 * n + es * n
    for j in range(1, m_eff):
        b += (j + 1) * es * n
    return b


def phi_bytes(n, es, m_eff):
    """Algorithmic bytes of the operator launches of one solve whose W is
    formed in memory: step j reads V_j and writes W = Phi(V_j)."""
    return m_eff * (es * n + 4 * n)


def gk_tile_bytes(n, es, m_eff):
    """Algorithmic bytes of the tile launches of one sketched Golub-Kahan
    solve: sketch of R0 and U_1 = R0/beta_1 (read R0 twice, write U_1);
    column c forms V_c (reads V_{c-1} from c = 2, writes V_c) and, before the
    last column, U_{c+1} (reads U_c, writes U_{c+1}); the assembly reads
    V_1..V_m and writes X.  The read of W is not counted (the method does not
    need W in memory)."""
    b = 2 * 4 * n + es * n
    for c in range(1, m_eff + 1):
        b += (es * n if c >= 2 else 0) + es * n
        if c < m_eff:
            b += 2 * es * n
    return b + m_eff * es * n + 4 * n


def time_variant(plan, steps, warmup, rtg, torch, kind, bytes_of, pre=None, overlap=False):
    """Time `steps` batch solves; `pre` (the warm-start network forward that
    produces the X0 of the batch) runs inside every timed step.  Launches of
    kernel kind `kind` are bracketed by HIP events on their stream inside the
    library; `bytes_of(info)` gives the algorithmic bytes of those launches for
    one problem.  With `overlap` (a plan with a fallback and a `pre`) each step
    queues the solve and the copy of its flags, then the network of the next
    batch, and only then waits for the flags and queues the re-solves, so the
    GPU runs the network while the host waits; the network of the first batch
    runs in the warm-up, and every timed step still holds one network and one
    solve."""
    if overlap and pre is not None:
        def one():
            plan.begin()
            pre()
            plan.end()
        pre()
    else:
        def one():
            if pre is not None:
                pre()
            plan.run()
    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    rtg.event_timing_read()                     # clear
    rtg.event_timing_enable(1 << kind)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rtg.event_timing_enable(0)
    ev = rtg.event_timing_read()
    infos = plan.infos()
    kb = sum(bytes_of(inf) for inf in infos) * steps
    k_ms, k_launches = ev[kind]
    return {
        "seconds": t1 - t0,
        "k_ms": k_ms,
        "k_launches": k_launches,
        "k_bytes": kb,
        "infos": infos,
    }


def source_digest(kernel_src):
    """SHA-256 of a kernel source followed by the local headers it includes
    (recursively, each once, in the order met; paths relative to the
    including file), so that a change to a shared header also counts."""
    import hashlib
    import re
    h = hashlib.sha256()
    seen = set()

    def add(path):
        path = os.path.normpath(path)
        if path in seen or not os.path.exists(path):
            return
        seen.add(path)
        with open(path, "rb") as f:
            data = f.read()
        h.update(data)
        for inc in re.findall(rb'#include\s+"([^"]+)"', data):
            add(os.path.join(os.path.dirname(path), inc.decode()))

    add(os.path.join(ROOT, "paper_2603_00839_amd", "csrc", kernel_src))
    return h.hexdigest()


def recorded_traffic(kernel_src, variant, tune, batch):
    """HBM traffic per launch measured with rocprofv3 counters (FETCH_SIZE and
    WRITE_SIZE, scaled by a copy-kernel calibration) and recorded with the
    digest of the kernel source and its headers it was measured on
    (source_digest); None when either has changed since, when nothing was
    recorded, when the record is of another workload (the record names the
    variant and the batch size) or of other launch shapes than this run's
    (the record names them)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    sha = source_digest(kernel_src)
    ent = rec.get(kernel_src)
    if not ent or ent.get("source_sha256") != sha or ent.get("variant", "bf16_warm") != variant:
        return None
    if ent.get("batch") != batch:
        return None
    shapes = ent.get("launch_shapes")
    if not shapes or any(tune.get(k) != v for k, v in shapes.items()):
        return None
    return ent["bytes_per_launch"]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The float64 oracle on the host cores: problems 0 and 1 of the
    512x512x3 batch with every BLAS thread (the throughput figure), problem 0
    again with one BLAS thread, and problem 0 of the non-separable PSF batch
    (its RE only).  Returns the timings and the oracle's RE per problem."""
    import numpy as np
    from paper_2603_00839_amd import synth
    from oracle.operator import Operator, PSFOperator, make_observation
    from oracle.sketch import Sketch
    from oracle.gmres import rtg_gmres
    from oracle.metrics import relative_error
    from threadpoolctl import threadpool_info, threadpool_limits

    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])

    def oracle_solve(p, psf=False):
        op = PSFOperator(p.psf, p.b_band, p.dims) if psf else Operator(p.a1_band, p.a2_band, p.b_band)
        sk = Sketch(p.om1, p.om2, p.om3)
        C, delta, _ = make_observation(op, p.x_true, p.noise_dir, p.nu)
        t0 = time.perf_counter()
        r = rtg_gmres(op, sk, C.astype(np.float32), p.m, delta=delta, eta=1.01)
        return time.perf_counter() - t0, relative_error(p.x_true, r.X)

    re = {}
    t_all = 0.0
    for k in (0, 1):
        dt, re[k] = oracle_solve(synth.cfg2(k))
        t_all += dt
    with threadpool_limits(limits=1, user_api="blas"):
        t_one, _ = oracle_solve(synth.cfg2(0))
    _, re_psf = oracle_solve(synth.cfg2_psf(0), psf=True)
    return {"value": 2.0 / t_all, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": "2 of the 512x512x3 solves (problems 0 and 1), m=50, float64 NumPy oracle, "
                      f"{threads} BLAS threads",
            "one_thread": {"value": 1.0 / t_one, "unit": "solves/s", "cores": 1,
                           "sample": "problem 0 with one BLAS thread"},
            "cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
            "re": re, "re_psf0": re_psf}


def golden_re():
    """Stored oracle REs of the uneven batch and the video workload (written
    by tests/golden/make_oracle_re.py from the oracle alone)."""
    try:
        with open(GOLDEN_RE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def oracle_ratios(results, cb, gold):
    """RE of each variant over the float64 oracle's plain-solve RE on the
    sampled problems (the one-sided target: at most 1.01)."""
    out = {}
    cfg2_like = ("fp32_plain", "bf16_warm", "bf16_obs", "fp32_unsketched", "fp32_gk")
    for v, r in results.items():
        pairs = []
        if v in cfg2_like:
            pairs = [(r["re"][k], cb["re"][k]) for k in (0, 1) if k < len(r["re"])]
        elif v == "fp32_psf":
            pairs = [(r["re"][0], cb["re_psf0"])]
        elif v in ("fp32_uneven", "mixed_uneven", "mixed_uneven_persist") and gold:
            pairs = [(r["re"][int(k)], g["re"]) for k, g in gold["uneven"].items() if int(k) < len(r["re"])]
        elif v in ("fp32_video", "bf16_video") and gold:
            pairs = [(r["re"][0], gold["video"]["0"]["re"])]
        if pairs:
            out[v] = {"problems": len(pairs), "oracle_re": [o for _, o in pairs],
                      "max_re_over_oracle": max(g / o for g, o in pairs)}
    out["source"] = ("512x512x3 and PSF: oracle solves in the CPU-baseline leg; uneven batch and video: "
                     "tests/golden/oracle_re.json")
    return out


def tune_plan(plan, args, pre=None):
    """Launch shapes for this batch: picked by the library's autotuner
    (outside the timed region; X0 formed first where the step computes it),
    or the defaults with --no-autotune."""
    if args.tune:
        from paper_2603_00839_amd import rtg
        fields = dict(kv.split("=", 1) for kv in args.tune.split(",") if kv)
        plan.set_tune(rtg.make_tune(**{k: int(v) for k, v in fields.items()}))
        return {"autotuned": False, **plan.tune().as_dict()}
    if args.no_autotune:
        return {"autotuned": False, **plan.tune().as_dict()}
    if pre is not None:
        pre()
    t, ms = plan.autotune(reps=3)
    return {"autotuned": True, "loop_ms": ms, **t.as_dict()}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only: sharding over several GPUs "
                                   "(independent problems per GPU) is not implemented"}))
        sys.exit(2)
    import numpy as np
    import torch
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        x = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "copies": 3}), flush=True)
        return
    from paper_2603_00839_amd import rtg
    if not os.path.exists(rtg.LIB_PATH):
        from paper_2603_00839_amd import build_lib
        build_lib.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    B = args.batch
    op, probs = make_batch(B, dev)
    p0 = probs[0]["p"]
    I1, I2, J = p0.dims
    n = I1 * I2 * J

    # warm start: X0 = C + f(C) for the whole batch, recomputed in every timed step
    x0_kind = args.x0
    net = None
    if x0_kind == "learned":
        try:
            from paper_2603_00839_amd import warmstart
            net = warmstart.load_default(dev)
        except Exception as e:      # weights not trained yet
            print(f"[bench] learned warm start unavailable ({e}); using X0 = C", file=sys.stderr)
            x0_kind = "observation"
    Cbatch = torch.stack([q["C"] for q in probs]).contiguous()        # (B, 3, I2, I1)
    X0batch = Cbatch.clone()
    X0s = [X0batch[b] for b in range(B)]
    pre = (lambda: net.forward(Cbatch, out=X0batch)) if net is not None else None
    torch.cuda.synchronize()

    results = {}
    variants = [args.only] if args.only else list(VARIANTS)
    for v in variants:
        if v in ("fp32_video", "bf16_video"):
            # the video workload: float32 basis from X0 = 0, or a bfloat16
            # basis from X0 = C (the network is trained on colour images);
            # m = 80 steps (the discrepancy level is not reached within them)
            Bv = args.video_batch
            op_v, probs_v = make_video_batch(Bv, dev)
            nv = probs_v[0]["p"].dims[0] * probs_v[0]["p"].dims[1] * probs_v[0]["p"].dims[2]
            bfv = v == "bf16_video"
            prm = [rtg.make_params(80, rtg.BF16 if bfv else rtg.F32, delta=q["delta"], eta=1.01) for q in probs_v]
            plan = rtg.BatchPlan([op_v] * Bv, [q["sk"] for q in probs_v], [q["C"] for q in probs_v],
                                 [q["C"] for q in probs_v] if bfv else [None] * Bv, prm)
            tune = tune_plan(plan, args)
            if bfv:
                r = time_variant(plan, args.steps, args.warmup, rtg, torch, rtg.KIND_STEP,
                                 lambda inf: step_bytes(nv, 2, inf.iters))
                r["kernel"] = ("k_step", "k_step.hip", "Arnoldi step, bfloat16 basis, 256x256x64 videos")
            else:
                r = time_variant(plan, args.steps, args.warmup, rtg, torch, rtg.KIND_TILE,
                                 lambda inf: tile_bytes(nv, 4, inf.iters, False))
                r["kernel"] = ("k_tile", "k_tile.hip", "multi-AXPY + store + MFMA sketch, 256x256x64 videos")
            res = [rel_err(plan.outs[b], probs_v[b]["xt"]) for b in range(Bv)]
            r["solves_per_step"] = Bv
        elif v in ("fp32_uneven", "mixed_uneven", "mixed_uneven_persist"):
            probs_u = make_uneven_batch(dev)
            Bu = len(probs_u)
            bt = rtg.F32 if v == "fp32_uneven" else rtg.F32_BF16
            prm = [rtg.make_params(40, bt, delta=q["delta"], eta=1.01) for q in probs_u]
            plan = rtg.BatchPlan([q["op"] for q in probs_u], [q["sk"] for q in probs_u], [q["C"] for q in probs_u],
                                 [None] * Bu, prm)
            ns = [q["n"] for q in probs_u]
            it = {"i": 0}

            tune = tune_plan(plan, args)
            if v == "mixed_uneven_persist" and tune.get("persist") != 1:
                t = plan.tune()
                t.persist = 1
                plan.set_tune(t)
                tune = {**tune, "persist": 1}
            persist = tune.get("persist") == 1

            def bytes_u(inf, it=it):
                n_i = ns[it["i"] % Bu]
                b = arnoldi_bytes(n_i, 4, inf.iters) if persist else tile_bytes(n_i, 4, inf.iters, False)
                it["i"] += 1
                return b
            prod = "float32" if v == "fp32_uneven" else "bfloat16"
            if persist:
                r = time_variant(plan, args.steps, args.warmup, rtg, torch, rtg.KIND_PERSIST, bytes_u)
                r["kernel"] = ("k_persist", "k_persist.hip", "the Arnoldi process of all 256 uneven problems in "
                               "one persistent launch (operator, multi-AXPY + MFMA sketch, sketched Gram), "
                               "float32 basis, " + prod + " products")
            else:
                r = time_variant(plan, args.steps, args.warmup, rtg, torch, rtg.KIND_TILE, bytes_u)
                r["kernel"] = ("k_tile", "k_tile.hip", "multi-AXPY + store + MFMA sketch, float32 basis, "
                                                       + prod + " products, 256 uneven problems")
            res = [rel_err(plan.outs[b], probs_u[b]["xt"]) for b in range(Bu)]
            r["solves_per_step"] = Bu
        elif v == "fp32_psf":
            op_p, probs_p = make_psf_batch(B, dev)
            prm = [rtg.make_params(args.m, rtg.F32, delta=q["delta"], eta=1.01) for q in probs_p]
            plan = rtg.BatchPlan([op_p] * B, [q["sk"] for q in probs_p], [q["C"] for q in probs_p], [None] * B, prm)
            tune = tune_plan(plan, args)
            r = time_variant(plan, args.steps, args.warmup, rtg, torch, rtg.KIND_PHI,
                             lambda inf: phi_bytes(n, 4, inf.iters))
            r["kernel"] = ("k_phi", "k_operator.hip", "2-D stencil of a general PSF + channel mix (float32)")
            res = [rel_err(plan.outs[b], probs_p[b]["xt"]) for b in range(B)]
        elif v == "fp32_gk":
            prm = [rtg.make_params(args.m, rtg.F32, delta=q["delta"], eta=1.01, method=rtg.METHOD_GOLUB_KAHAN)
                   for q in probs]
            plan = rtg.BatchPlan([op] * B, [q["sk"] for q in probs], [q["C"] for q in probs], [None] * B, prm)
            tune = tune_plan(plan, args)
            r = time_variant(plan, args.steps, args.warmup, rtg, torch, rtg.KIND_TILE,
                             lambda inf: gk_tile_bytes(n, 4, inf.iters))
            r["kernel"] = ("k_tile", "k_tile.hip", "one-term AXPY + store + MFMA mode-1/2 sketch "
                                                   "(Golub-Kahan, float32 basis)")
        elif v == "fp32_unsketched":
            # the same solve with the identity sketch: Frobenius inner products of
            # the full tensors (the unsketched global GMRES the method improves on)
            sk_id = rtg.setup_sketch(I1, I2, J)
            prm = [rtg.make_params(args.m, rtg.F32, delta=q["delta"], eta=1.01) for q in probs]
            plan = rtg.BatchPlan([op] * B, [sk_id] * B, [q["C"] for q in probs], [None] * B, prm)
            tune = tune_plan(plan, args)
            r = time_variant(plan, args.steps, args.warmup, rtg, torch, rtg.KIND_GRAM,
                             lambda inf: frob_bytes(n, 4, inf.iters))
            r["kernel"] = ("k_gram", "k_gram.hip", "Frobenius inner products of the full tensors "
                                                   "(float32 basis, identity sketch)")
        elif v == "fp32_plain":
            prm = [rtg.make_params(args.m, rtg.F32, delta=q["delta"], eta=1.01) for q in probs]
            plan = rtg.BatchPlan([op] * B, [q["sk"] for q in probs], [q["C"] for q in probs], [None] * B, prm)
            tune = tune_plan(plan, args)
            r = time_variant(plan, args.steps, args.warmup, rtg, torch, rtg.KIND_TILE,
                             lambda inf: tile_bytes(n, 4, inf.iters, False))
            r["kernel"] = ("k_tile", "k_tile.hip", "multi-AXPY + store + MFMA mode-1/2 sketch (float32 basis)")
        else:
            # bf16_warm (the network's X0, recomputed in every timed step) or
            # bf16_obs (X0 = C); failed warm starts re-solved by the plain solver
            obs = v == "bf16_obs"
            prm = [rtg.make_params(args.m_warm, rtg.BF16, delta=q["delta"], eta=1.01,
                                   stop_res=(1.01 * q["delta"] if args.warm_stop == "discrepancy" else 0.0))
                   for q in probs]
            x0v = [q["C"] for q in probs] if obs else X0s
            plan = rtg.BatchPlan([op] * B, [q["sk"] for q in probs], [q["C"] for q in probs], x0v, prm,
                                 fallback=(FALLBACK_M, rtg.F32))
            tune = tune_plan(plan, args, None if obs else pre)

            def warm_bytes(inf):
                # a problem re-solved by the plain solver counts the step launches
                # of its warm attempt only (the re-solve runs the tile kernel)
                return step_bytes(n, 2, args.m_warm if inf.flags & rtg.FLAG_FALLBACK else inf.iters)
            r = time_variant(plan, args.steps, args.warmup, rtg, torch, rtg.KIND_STEP, warm_bytes,
                             pre=None if obs else pre, overlap=args.overlap == "on")
            r["kernel"] = ("k_step", "k_step.hip", "Arnoldi step: operator per tile + multi-AXPY + store + "
                                                   "dual MFMA sketch (bfloat16 basis)")
            r["fallbacks_per_step"] = plan.n_fallback
            r["overlap"] = args.overlap == "on" and not obs
        if v not in ("fp32_psf", "fp32_uneven", "mixed_uneven", "mixed_uneven_persist", "fp32_video", "bf16_video"):
            res = [rel_err(plan.outs[b], probs[b]["xt"]) for b in range(B)]
        r["tune"] = tune
        r["re"] = res
        r["re_mean"] = float(np.mean(res))
        r["re_p0"] = res[0]
        r["iters_mean"] = float(np.mean([i.iters for i in r["infos"]]))
        r["flags"] = sorted({i.flags for i in r["infos"]})
        fc = {}
        for i in r["infos"]:
            fc[str(i.flags)] = fc.get(str(i.flags), 0) + 1
        r["flag_counts"] = fc
        r["solves_per_s"] = r.get("solves_per_step", B) * args.steps / r["seconds"]
        r["ms_per_step"] = 1e3 * r["seconds"] / args.steps
        results[v] = r
        del plan
        torch.cuda.empty_cache()

    if args.headline == "auto":
        head = "bf16_warm" if (x0_kind == "learned" and "bf16_warm" in results) else variants[0]
    else:
        head = args.headline
    if head not in results:
        head = variants[0]
    H = results[head]
    gbs = H["k_bytes"] / (H["k_ms"] * 1e-3) / 1e9 if H["k_ms"] > 0 else 0.0
    bpl = H["k_bytes"] / max(H["k_launches"], 1)
    traffic = recorded_traffic(H["kernel"][1], head, H["tune"], B)
    out = {
        "metric": METRIC,
        "value": H["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": H["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32_plain" else "bf16",
        "data": "synthetic",
        "config": {
            "workload": "cfg2: 512x512x3 colour deblurring (200 rectangles + Gaussian random field, "
                        "sigma 2.5, r 8, nu 1e-3), sketch 64x64x3, discrepancy mu",
            "problems_per_step": B, "m": args.m if head == "fp32_plain" else args.m_warm,
            "variant": head, "x0": "zero" if head == "fp32_plain" else x0_kind,
            "stop": "m steps" if head == "fp32_plain" else
                    ("m steps" if args.warm_stop == "fixed" else "LS residual <= eta*delta, at most m steps"),
            "x0_in_timed_region": head != "fp32_plain",
        },
        "roofline": {
            "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": f"{H['kernel'][0]} ({H['kernel'][2]})",
            "launches": H["k_launches"],
            "avg_launch_us": 1e3 * H["k_ms"] / max(H["k_launches"], 1),
            "bytes_per_launch": bpl,
        },
        "launch_shapes": H["tune"],
        "variants": {k: {"solves_per_s": v["solves_per_s"], "ms_per_step": v["ms_per_step"],
                         "re_mean": v["re_mean"], "re_problem0": v["re_p0"], "iters_mean": v["iters_mean"],
                         "flags": v["flags"], "flag_counts": v["flag_counts"],
                         "fallbacks_per_step": v.get("fallbacks_per_step"),
                         "overlap": v.get("overlap"),
                         "kernel": v["kernel"][0], "tune": v["tune"],
                         "kernel_gbs": (v["k_bytes"] / (v["k_ms"] * 1e-3) / 1e9 if v["k_ms"] > 0 else 0.0)}
                     for k, v in results.items()},
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline()
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "one_thread",
                                                  "cpu_count", "cpu_model")}
        out["oracle_re"] = oracle_ratios(results, cb, golden_re())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
