"""What the trained period-proposal network gains over a ranking without it,
on the 90-day stand-in workload (`learned.training_curve`: 4,409 points at
29.4-minute cadence, sigma 100-400 ppm, 70 % with one transit; a grid of
10,482 Ofir periods and 12 durations): the network is trained on 4,096
curves labelled by the library's full-grid search (1,500 Adam steps of batch
128) and scored on 128 held-out curves.  The bar: its top 32 of 512 log-period bins hold the held-out curves'
full-grid best period more often than the 32 bins most frequent among the
training labels (the prior-only ranking), by at least 5 points; the pruned
search with its full-grid fallback is faster than the full grid.  Training
and search are deterministic, so the figures printed repeat exactly."""
import pytest

from paper_2607_00348_amd import learned

pytestmark = pytest.mark.gpu


def test_network_beats_prior_ranking_on_held_out_curves():
    print("[learned] 4096 training curves, 128 held out", flush=True)
    res = learned.run(n_train=4096, n_test=128, steps=1500, k=32, seed=0, batch=128, lr=3e-3,
                      log=lambda m: print(f"[learned] {m}", flush=True))
    print(f"[learned] recall@32 network {res['recall_at_k_net']:.3f} vs prior {res['recall_at_k_prior']:.3f}; "
          f"final recall {res['recall_best_period']:.3f} with {res['fallback_fraction']:.2f} fallback; "
          f"speed-up {res['speedup']:.2f}x; final loss {res['final_loss']:.3f}", flush=True)
    assert res["recall_at_k_net"] >= res["recall_at_k_prior"] + 0.05
    assert res["speedup"] > 1.0
