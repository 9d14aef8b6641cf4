"""The shipped start-proposal network (paper_2104_07146_amd/data/start_mlp.npz)
checked without a GPU: the file loads without unpickling, its sizes match the
network, its training report shows the validation loss fell, and on fields
drawn at known parameters (2048 uniform points, parameters from the training
ranges, the dense oracle's sampler) the network, evaluated by the oracle's
features and forward pass with the shipped weights and normalisation,
predicts the standardised log-parameters far better than their training
mean does (whose squared error is about 1)."""
import json
import os

import numpy as np

import synth
from oracle import dense, learned

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2104_07146_amd", "data",
                       "start_mlp.npz")


def test_shipped_weights_predict_the_parameters():
    d = np.load(WEIGHTS, allow_pickle=False)
    params, norm = d["params"].astype(np.float64), d["norm"].astype(np.float64)
    assert params.shape == (learned.n_params(),) and norm.shape == (74,)
    report = json.loads(str(d["report"]))
    assert report["val_mse"] < report["val_mse_first"]
    mu_x, sd_x, mu_y, sd_y = norm[:33], norm[33:66], norm[66:70], norm[70:74]
    assert np.all(sd_x > 0) and np.all(sd_y > 0)
    rng = synth.rng_for(synth.W_TESTS, 995)
    t_true, t_pred = [], []
    for _ in range(12):
        pts = synth.uniform_points(2048, 2, rng)
        theta = synth.batch_theta(rng)
        z = dense.sample(pts, theta, synth.standard_normal(2048, rng))
        x = learned.standardise(learned.variogram_features(pts, z), mu_x, sd_x)
        _, y = learned.forward(params, x[None, :])
        t_true.append((np.log(theta) - mu_y) / sd_y)
        t_pred.append(y[0])
    t_true, t_pred = np.array(t_true), np.array(t_pred)
    mse = float(np.mean((t_pred - t_true) ** 2))
    baseline = float(np.mean(t_true ** 2))
    print(f"standardised log-parameter MSE {mse:.3f} (training mean: {baseline:.3f})")
    assert mse <= 0.4 and mse <= 0.5 * baseline
