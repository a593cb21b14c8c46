"""The MC-truth report (paper_2106_03636_amd/mctruth.py) on hand-built
outputs, and against the pins' own efficiency count on oracle results."""
import numpy as np

from conftest import cached_event, cached_oracle
from paper_2106_03636_amd import mctruth


def test_hand_built_match_fake_clone():
    # unit 0: particle 0 has 50 clusters (ids 0..49), particle 1 has 45 (50..94),
    # particle 2 has 10 (95..104, not findable); 5 noise clusters (105..109)
    label = np.array([0] * 50 + [1] * 45 + [2] * 10 + [-1] * 5)
    pt = np.array([0.4, 3.0, 1.0])
    tracks = [list(range(0, 45)) + [105, 106, 107, 108, 109],   # 45/50 = 0.9 of particle 0: matched
              list(range(50, 90)) + list(range(95, 100)),       # 40/45 = 0.889 of particle 1: fake
              list(range(10, 30))]                              # particle 0 again: a clone
    first = np.cumsum([0] + [len(t) for t in tracks[:-1]])
    r = mctruth.report(label, [0, len(label)], pt, first, [len(t) for t in tracks], np.concatenate(tracks))
    assert r["findable"] == 2 and r["tracks"] == 3
    assert r["efficiency"] == 0.5 and abs(r["fake_rate"] - 1 / 3) < 1e-12 and r["clone_rate"] == 0.5
    byb = {b["pt_lo"]: b for b in r["vs_pt"]}
    assert byb[0.3]["efficiency"] == 1.0 and byb[2.0]["efficiency"] == 0.0


def test_agrees_with_the_pins_count():
    import test_oracle_pins as pins
    for name in ("pp_sector", "pbpb_central"):
        ev, o = cached_event(name), cached_oracle(name)
        r = mctruth.report(ev.label, ev.unit_offsets, ev.tracks.pt, o["track_first_hit"], o["track_n_hits"],
                           o["track_hits"], pt_min=0.2)
        eff, fake, nf = pins._efficiency(ev, o)
        assert r["findable"] == nf and abs(r["efficiency"] - eff) < 1e-12 and abs(r["fake_rate"] - fake) < 1e-12
