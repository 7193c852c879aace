"""Adam on (sigma_s, g) of the fog layer with the adjoint kernel.

A time-resolved image of this layer constrains the reduced scattering
coefficient sigma_s (1 - g) sharply and the split between sigma_s and g only
weakly (the diffusion approximation depends on sigma_s and g only through
sigma_s (1 - g), Eq. (9), and the measured gradient along sigma_s (1 - g) =
const is below its noise at 2^26 paths), so the checks are that the fit
recovers sigma_s (1 - g) and stays a valid medium; where along the valley
the iterates end depends on the random streams (and the reported loss, the
squared residual of one noisy render, is dominated by render noise).  The
adjoint itself is checked against the oracle and finite differences
elsewhere."""
import numpy as np
import pytest
import torch

from paper_2402_03106_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_03106_amd import darts
    darts.lib()
    return darts


def test_fit_recovers_reduced_scattering(D):
    from paper_2402_03106_amd import inverse
    w = W.fog_slab_fit()
    tm, im = w["target_medium"], w["init_medium"]
    r = inverse.fit_medium(w, tm, im, steps=120, mode="da_only", lr=0.05, lr_final=0.01, n_paths=1 << 24)
    red_t = tm["sigma_s"] * (1 - tm["g"])
    red_i = im["sigma_s"] * (1 - im["g"])
    red = r["sigma_s"] * (1 - r["g"])
    loss = np.array([h["loss"] for h in r["history"]])
    print("estimate", r["sigma_s"], r["g"], "reduced", red, "target", red_t,
          "loss first 5", loss[:5].mean(), "last 20", loss[-20:].mean())
    assert abs(red / red_t - 1) < 0.1
    assert abs(red - red_t) < 0.5 * abs(red_i - red_t)
    assert all(np.isfinite([h["sigma_s"] for h in r["history"]]))
    assert r["sigma_s"] > 0 and abs(r["g"]) < 0.99
