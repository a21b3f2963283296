"""Training and evaluation of the learned zoom's window-proposal network.

The training data is made by the plain method itself: synthetic echoes of the
learned-zoom workload (100 pulses x 64 gates, code length 256, one line per
gate uniform in 1-15 MHz, per-gate SNR uniform in -25..-5 dB) are integrated
by the library at the coarse length N_c = 1024 (the network's input, as
features log(S / mean S)) and at the fine length N = 16384, whose peak bin,
divided by S = N / N_c, is the target position in coarse-bin units.  The
network trains with the library's own forward and backward kernels (FP32,
Adam); the weights are stored as raw little-endian float32 next to this file
together with a JSON record of how they were made.

    python -m paper_2311_18737_amd.zoom_training train --gates 200000
    python -m paper_2311_18737_amd.zoom_training eval

Echo drawing runs on the host in a pool of worker processes that is forked
before the GPU is first touched; the workers never use the GPU.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "zoom_net.f32")
RECORD = os.path.join(HERE, "weights", "zoom_net.json")

COARSE = 1024
TRAIN_SEED0 = 1            # training datasets use seeds 1, 2, ...
EVAL_SEED0 = 1_000_000     # evaluation datasets never overlap them


def _root():
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    return root


def workload(n_pulses: int = 100):
    _root()
    from synth import CONFIGS

    return CONFIGS["zoom"].replace(n_pulses=n_pulses)


def _draw(args):
    """Worker: one dataset's samples and codes (host memory only)."""
    cfg, seed = args
    _root()
    from synth import make_dataset

    d = make_dataset(cfg, seed, cache_dir=None)
    return seed, d.samples, d.tx


def load_weights(path: str = WEIGHTS) -> np.ndarray:
    from . import _lib

    p = np.fromfile(path, dtype="<f4")
    if p.shape != (_lib.ISPL_NET_PARAMS,):
        raise ValueError(f"{path}: expected {_lib.ISPL_NET_PARAMS} float32 values, got {p.shape}")
    return p


class SpectrumMaker:
    """Coarse features and fine peak bins of whole datasets through the library."""

    def __init__(self, cfg, net, device: int = 0):
        import torch

        from .context import Context

        self.torch = torch
        self.cfg = cfg
        self.dev = torch.device("cuda", device)
        geo = dict(code_len=cfg.code_len, n_gates=cfg.n_gates, gate_step=cfg.gate_step,
                   first_gate=cfg.first_gate, pulse_stride=cfg.pulse_stride,
                   sample_type=cfg.sample_type, max_pulses=cfg.n_pulses, device=device)
        self.coarse = Context(fft_len=COARSE, **geo)
        self.fine = Context(fft_len=cfg.fft_len, **geo)
        self.net = net
        self.S = cfg.fft_len // COARSE

    def upload(self, samples, tx):
        t = self.torch
        return (t.from_numpy(np.ascontiguousarray(samples)).to(self.dev),
                t.from_numpy(np.ascontiguousarray(tx)).to(self.dev))

    def features(self, xs, xt):
        sc = self.coarse.integrate_spectra(xs, xt)
        return self.net.features(sc), sc

    def fine_peaks(self, xs, xt):
        sf = self.fine.integrate_spectra(xs, xt)
        bins, _ = self.fine.find_plasma_line(sf)
        return bins, sf

    def close(self):
        self.coarse.close()
        self.fine.close()


def make_training_set(n_gates_total: int, pool, maker, seed0: int, log=print):
    """features [M][1024] (device) and targets [M] (device, coarse units)."""
    torch = maker.torch
    cfg = maker.cfg
    n_sets = math.ceil(n_gates_total / cfg.n_gates)
    feats = torch.empty((n_sets * cfg.n_gates, COARSE), dtype=torch.float32, device=maker.dev)
    targ = torch.empty(n_sets * cfg.n_gates, dtype=torch.float32, device=maker.dev)
    t0 = time.time()
    jobs = ((cfg, seed0 + i) for i in range(n_sets))
    for i, (seed, samples, tx) in enumerate(pool.imap(_draw, jobs, chunksize=4)):
        xs, xt = maker.upload(samples, tx)
        f, _ = maker.features(xs, xt)
        bins, _ = maker.fine_peaks(xs, xt)
        rows = slice(i * cfg.n_gates, (i + 1) * cfg.n_gates)
        feats[rows] = f
        targ[rows] = bins.to(torch.float32) / maker.S
        if (i + 1) % 200 == 0 or i + 1 == n_sets:
            torch.cuda.synchronize()
            log(f"  data: {i + 1}/{n_sets} datasets ({(i + 1) * cfg.n_gates} gates), "
                f"{time.time() - t0:.1f} s")
    return feats, targ


def train(args):
    import multiprocessing as mp

    cfg = workload()
    # fork the echo-drawing workers before anything touches the GPU
    pool = mp.get_context("fork").Pool(args.workers)
    import torch

    from .context import Net

    torch.manual_seed(args.seed)
    net = Net(args.batch)
    net.set_params(he_init(args.seed))
    maker = SpectrumMaker(cfg, net)
    print(f"drawing {args.gates} training gates ({cfg.n_pulses} pulses each)", flush=True)
    feats, targ = make_training_set(args.gates, pool, maker, TRAIN_SEED0)
    pool.close()
    pool.join()
    M = feats.shape[0]
    steps_per_epoch = M // args.batch
    total = steps_per_epoch * args.epochs
    gen = torch.Generator(device=maker.dev)
    gen.manual_seed(args.seed)
    loss_buf = torch.empty(1, dtype=torch.float32, device=maker.dev)
    t0 = time.time()
    hist = []
    step = 0
    for ep in range(args.epochs):
        perm = torch.randperm(M, device=maker.dev, generator=gen)
        run = torch.zeros(1, dtype=torch.float64, device=maker.dev)
        for b in range(steps_per_epoch):
            idx = perm[b * args.batch:(b + 1) * args.batch]
            xb = feats.index_select(0, idx)
            ub = targ.index_select(0, idx)
            # linear warm-up over 200 steps, then cosine decay to 1 % of lr
            warm = min(1.0, (step + 1) / 200.0)
            cos = 0.5 * (1 + math.cos(math.pi * step / max(1, total)))
            lr = args.lr * warm * (0.01 + 0.99 * cos)
            net.train_step(xb, ub, lr, loss=loss_buf)
            run += loss_buf
            step += 1
        mean_loss = float(run.item()) / steps_per_epoch
        hist.append(mean_loss)
        print(f"  epoch {ep + 1}/{args.epochs}: mean loss {mean_loss:.4f}, "
              f"{time.time() - t0:.1f} s", flush=True)
    params = net.get_params()
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    params.astype("<f4").tofile(args.out)
    rec = {"workload": {"n_pulses": cfg.n_pulses, "n_gates_per_set": cfg.n_gates,
                        "code_len": cfg.code_len, "coarse_len": COARSE, "fine_len": cfg.fft_len,
                        "f_line_hz": list(cfg.f_peak_hz), "snr_db": list(cfg.snr_db_range)},
           "training_gates": int(M), "training_seeds": [TRAIN_SEED0, TRAIN_SEED0 + M // cfg.n_gates - 1],
           "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "init_seed": args.seed,
           "epoch_mean_loss": hist, "train_seconds": round(time.time() - t0, 1),
           "command": "python -m paper_2311_18737_amd.zoom_training train "
                      f"--gates {args.gates} --epochs {args.epochs} --batch {args.batch} "
                      f"--lr {args.lr} --seed {args.seed}"}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {args.out}", flush=True)
    maker.close()
    net.close()
    return params


def he_init(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, in the library's parameter order."""
    rng = np.random.default_rng([2311, 18737, 77, seed])
    parts = []
    for cin, cout in ((1, 32), (32, 32), (32, 32), (32, 1)):
        parts.append(rng.standard_normal(cout * cin * 7) * math.sqrt(2.0 / (cin * 7)))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


def evaluate(params, n_sets: int = 16, threshold: float = 0.9, window_bins: int = 256,
             seed0: int = EVAL_SEED0, log=None):
    """Learned zoom on held-out datasets against the full-resolution peaks.

    Returns per-gate arrays: full-FFT peak (the reference), learned-zoom peak,
    whether the gate was zoomed, its confidence, and the coarse-argmax
    heuristic's peak (window on the coarse spectrum's argmax, always zoomed).
    """
    import torch

    from .context import LearnedZoom, Net, Zoom

    _root()
    from synth import make_dataset

    cfg = workload()
    net = Net(1)
    net.set_params(params)
    maker = SpectrumMaker(cfg, net)
    lz = LearnedZoom(net, code_len=cfg.code_len, fft_len=cfg.fft_len, n_gates=cfg.n_gates,
                     gate_step=cfg.gate_step, first_gate=cfg.first_gate,
                     pulse_stride=cfg.pulse_stride, sample_type=cfg.sample_type,
                     max_pulses=cfg.n_pulses, window_bins=window_bins, threshold=threshold)
    hz = Zoom(maker.fine, window_bins, "fp16x3")
    all_gates = torch.arange(cfg.n_gates, dtype=torch.int32, device=maker.dev)
    count = torch.tensor([cfg.n_gates], dtype=torch.int32, device=maker.dev)
    out = {k: [] for k in ("full_fft", "learned", "zoomed", "confidence", "heuristic", "snr_db",
                           "truth")}
    for i in range(n_sets):
        d = make_dataset(cfg, seed0 + i, cache_dir=None)
        xs, xt = maker.upload(d.samples, d.tx)
        full_fft, _ = maker.fine_peaks(xs, xt)
        bins, _ = lz.peaks(xs, xt)
        torch.cuda.synchronize()
        v = lz.view()
        conf = v["confidence"].cpu().numpy().copy()
        n_zoom = int(v["counts"][0].item())
        zl = v["zoom_list"][:n_zoom].cpu().numpy()
        zoomed = np.zeros(cfg.n_gates, bool)
        zoomed[zl] = True
        # heuristic: window centred on the coarse spectrum's argmax, always zoomed
        sc = v["coarse_spectra"]
        m = torch.argmax(sc, dim=1).to(torch.int64)
        hstart = ((m * maker.S - window_bins // 2) % cfg.fft_len).to(torch.int32)
        hs = hz.spectra(xs, xt, hstart)
        hb, _ = hz.find_peaks(hs, hstart, (all_gates, count))
        out["full_fft"].append(full_fft.cpu().numpy())
        out["learned"].append(bins.cpu().numpy())
        out["zoomed"].append(zoomed)
        out["confidence"].append(conf)
        out["heuristic"].append(hb.cpu().numpy())
        out["snr_db"].append(10 * np.log10(d.rho_gate))
        out["truth"].append(d.truth_bin())
        if log:
            log(f"  eval set {i + 1}/{n_sets}: zoomed {n_zoom}/{cfg.n_gates}")
    hz.close()
    lz.close()
    maker.close()
    net.close()
    return {k: np.concatenate(v) for k, v in out.items()}


def summarise(ev: dict, fine_len: int = 16384) -> dict:
    def err(a, b):
        d = np.mod(a.astype(np.int64) - b.astype(np.int64), fine_len)
        return np.minimum(d, fine_len - d)

    e_learn = err(ev["learned"], ev["full_fft"])
    e_heur = err(ev["heuristic"], ev["full_fft"])
    z = ev["zoomed"]
    # the heuristic restricted to the gates the network zooms (same split)
    return {
        "gates": int(z.size),
        "zoomed_fraction": float(z.mean()),
        "learned_within_1_bin": float(np.mean(e_learn <= 1)),
        "learned_within_1_bin_zoomed": float(np.mean(e_learn[z] <= 1)) if z.any() else None,
        "heuristic_within_1_bin": float(np.mean(e_heur <= 1)),
        "heuristic_within_1_bin_on_zoomed": float(np.mean(e_heur[z] <= 1)) if z.any() else None,
        "heuristic_within_1_bin_on_fallback": (float(np.mean(e_heur[~z] <= 1))
                                              if (~z).any() else None),
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--gates", type=int, default=200_000)
    t.add_argument("--epochs", type=int, default=8)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--workers", type=int, default=12)
    t.add_argument("--out", default=WEIGHTS)
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--sets", type=int, default=16)
    e.add_argument("--threshold", type=float, default=0.9)
    a = ap.parse_args(argv)
    if a.cmd == "train":
        train(a)
    else:
        ev = evaluate(load_weights(a.weights), n_sets=a.sets, threshold=a.threshold,
                      log=lambda m: print(m, flush=True))
        print(json.dumps(summarise(ev), indent=1), flush=True)


if __name__ == "__main__":
    main()
