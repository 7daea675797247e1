"""The stored oracle run of the shedding cylinder against the paper's values for
Re = 100 (Table high-Re: C_d = 1.336 +- 0.008, C_l = +-0.304, St = 0.169 on a
2048 x 1024 grid with D = 40). This build's channel is half as wide (blockage
7.8% instead of 3.9%), which raises drag and shedding frequency, so the check
is a band, not parity."""
import json
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cylinder_re100_oracle.json")


def test_oracle_shedding_in_the_papers_band():
    g = json.load(open(GOLDEN))["summary"]
    assert 1.25 <= g["cd_mean"] <= 1.55
    assert 0.155 <= g["st"] <= 0.185
    assert 0.25 <= g["cl_amp"] <= 0.45
    assert g["cd_amp"] < 0.05            # drag oscillates at twice St with small amplitude


WAKE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "steady_wake_oracle.json")
# paper, Table low-Re: C_d, L_s/D, theta_s (degrees) at Re = 20 and 40
PAPER_LOW_RE = {20.0: (2.09, 0.93, 43.0), 40.0: (1.55, 2.25, 52.9)}


def test_oracle_steady_wakes_near_the_papers_table():
    """The stored oracle runs of the steady cylinder wakes (noise-free, 60k steps)
    are steady (drag changes by < 1e-4 over the last 1000 steps), symmetric (lift
    ~ 0) and near the paper's values. This channel has twice the paper's blockage
    (7.8% instead of 3.9%), which raises the drag; recirculation length and
    separation angle agree within 6% and 4 degrees."""
    for c in json.load(open(WAKE))["cases"]:
        cd_p, ls_p, th_p = PAPER_LOW_RE[c["re"]]
        assert abs(c["cd"] - c["cd_1000_before"]) <= 1e-4 * c["cd"]
        assert abs(c["cl"]) <= 1e-10
        assert cd_p <= c["cd"] <= 1.15 * cd_p
        assert abs(c["ls_over_d"] - ls_p) <= 0.06 * ls_p
        assert abs(c["theta_s_deg"] - th_p) <= 4.0
