"""Admission policy of the server (host logic, no GPU)."""
from types import SimpleNamespace as NS

from paper_1311_2661_amd.serve import admit


def reqs(*spec):
    return [NS(ws_bytes=b, kind=k) for b, k in spec]


def test_first_fit_in_arrival_order():
    w = reqs((50, "vc"), (80, "mc"), (30, "mis"), (40, "vc"))
    # 100 bytes: 50 fits, 80 does not, 30 fits, 40 no longer fits
    assert admit(w, 100, {"ones": 8, "signed": 8}) == [0, 2]


def test_slots_limit_per_group():
    w = reqs((1, "vc"), (1, "mis"), (1, "vc"), (1, "mc"))
    slots = {"ones": 2, "signed": 1}
    assert admit(w, 10**9, slots) == [0, 1, 3]
    assert slots == {"ones": 0, "signed": 0}


def test_nothing_fits_means_wait_not_drop():
    w = reqs((500, "vc"), (600, "mc"))
    assert admit(w, 100, {"ones": 4, "signed": 4}) == []
    assert len(w) == 2


def test_budget_is_never_exceeded():
    import random
    rnd = random.Random(0)
    for _ in range(200):
        w = reqs(*[(rnd.randint(1, 100), rnd.choice(["vc", "mis", "mc"])) for _ in range(20)])
        free = rnd.randint(0, 400)
        picked = admit(w, free, {"ones": 5, "signed": 5})
        assert sum(w[k].ws_bytes for k in picked) <= free


def test_hold_blocks_newer_requests():
    w = reqs((10, "vc"), (10, "mis"), (10, "vc"))
    assert admit(w, 100, {"ones": 8}, hold_from=1) == [0]
    assert admit(w, 100, {"ones": 8}, hold_from=0) == []
