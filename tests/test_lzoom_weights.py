"""The committed network weights of the learned zoom, checked on the CPU with
the FP64 oracles only: the record matches the file, and the oracle network
with these weights, fed coarse spectra computed by the oracle from held-out
synthetic echoes, proposes windows that hold each strong gate's line."""

import json
import os

import numpy as np

import oracle.ispl_cnn as cnn
import oracle.ispl_lzoom as lzo
from oracle import integrate_spectra
from synth import CONFIGS, make_dataset

WDIR = os.path.join(os.path.dirname(__file__), "..", "paper_2311_18737_amd", "weights")


def load():
    p = np.fromfile(os.path.join(WDIR, "zoom_net.f32"), dtype="<f4")
    rec = json.load(open(os.path.join(WDIR, "zoom_net.json")))
    return p, rec


def test_weights_file_and_record():
    p, rec = load()
    assert p.shape == (cnn.N_PARAMS,) and np.all(np.isfinite(p))
    assert rec["training_gates"] >= 200_000
    assert rec["workload"]["coarse_len"] == 1024 and rec["workload"]["fine_len"] == 16384
    assert rec["epoch_mean_loss"][-1] < rec["epoch_mean_loss"][0]


def test_oracle_network_with_trained_weights_finds_the_lines():
    p, _ = load()
    cfg = CONFIGS["zoom"]
    d = make_dataset(cfg, 1_000_777, cache_dir=None)  # held out: training used seeds < 4000
    S = integrate_spectra(d.samples, d.tx, n_gates=cfg.n_gates, gate_step=cfg.gate_step,
                          first_gate=0, fft_len=1024, tx_per_pulse=True)
    X = cnn.features(S)
    truth = d.truth_bin(cfg.fft_len)
    snr = 10 * np.log10(d.rho_gate)
    inside, confident = [], []
    for g in range(cfg.n_gates):
        logits, _ = cnn.forward(p.astype(np.float64), X[g])
        start, conf, zoom, _, _ = lzo.select_window(logits, cfg.fft_len, 256, 0.9)
        off = (truth[g] - start) % cfg.fft_len
        inside.append(off < 256)
        confident.append(zoom)
    inside, confident = np.array(inside), np.array(confident)
    strong = snr > -20
    assert strong.sum() >= 20
    assert inside[strong].all()           # every strong gate's line lies in its window
    assert confident[strong].mean() >= 0.95
    # and where the network is confident, the window holds the line
    assert inside[confident].mean() >= 0.98
