"""The learned coarse-grid corrector end to end on a small driven domain: data from
fine trajectories, training, and the gain test (the corrected coarse run is closer
to the fine run than the plain coarse run from the same start).

A trained network has no oracle; what is checked is that training on the
solver's own residuals makes the coarse solution better, the property the
pipeline exists for.  Sizes are small (fine 256^2, coarse 64^2) so the whole test
takes seconds; the full-size measurement is the surrogate module's report.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_corrector_beats_plain_coarse_steps():
    from paper_2411_18341_amd import surrogate
    pl = surrogate.Pipeline(n_fine=256)
    X, R = pl.generate(list(range(10000, 10024)), snapshots=8, every=100, log=lambda s: None)
    assert np.isfinite(X.cpu().numpy()).all() and np.isfinite(R.cpu().numpy()).all()
    net, hist, _ = pl.train(X, R, epochs=6, batch=16, lr=1e-3, log=lambda s: None)
    assert hist[-1] < hist[0]
    res = pl.evaluate(net, list(range(20000, 20006)), t_start=800, horizons=(8, 64), log=lambda s: None)
    for H, r in res.items():
        plain, corr = r["plain_256"]["rel_l2_density"], r["corrected_256"]["rel_l2_density"]
        print(f"{H} fine steps: plain {plain:.4g}, corrected {corr:.4g}")
        assert corr < plain, H
    net.close()
