"""GPU parity when the recompute list overflows.

The list of pairs to recompute in int32 (Section 4.2: a score that reaches the int16
ceiling is recomputed exactly) holds a bounded number of entries (SW_KNOB_FLAG_CAP).
Pairs beyond it are marked in the scores and recomputed by a pass over every pair.  With
a capacity of one or a few entries, every path that flags pairs (one query per lane, two
queries per lane, two-pair intra-task items, long sequences, a captured plan) must still
give the oracle's scores.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1702_07195_amd import swmi, synth

pytestmark = pytest.mark.gpu

ALPHA = len(synth.ALPHABET)


def _say(msg):
    print(msg, flush=True)


class _Knobs:
    def __init__(self, **kv):
        self.kv = {getattr(swmi, "SW_KNOB_" + k.upper()): v for k, v in kv.items()}

    def __enter__(self):
        self.old = {k: swmi.get_knob(k) for k in self.kv}
        for k, v in self.kv.items():
            swmi.set_knob(k, v)

    def __exit__(self, *exc):
        for k, v in self.old.items():
            swmi.set_knob(k, v)


def _oracle(q, db, sm, go, ge):
    return oracle.search(q, db.residues, db.offsets, sm, go, ge)


@pytest.fixture(scope="module")
def mixed_db():
    # short sequences, two groups' worth of mid-length ones and three longer than the
    # intra-task threshold of this test (kept out of the groups at load time)
    rng = np.random.Generator(np.random.PCG64(3131))
    lengths = np.concatenate([rng.integers(0, 300, 150), rng.integers(800, 1500, 20),
                              [2600, 3100, 2900]])
    return synth.db_from_lengths(rng, lengths)


@pytest.mark.parametrize("route", [1 << 30, 0, 1])
@pytest.mark.parametrize("cap", [1, 7])
def test_recompute_everything_through_a_tiny_list(mixed_db, route, cap):
    rng = np.random.Generator(np.random.PCG64(41 + cap))
    qs = [synth.residues(rng, 700), synth.residues(rng, 90)]
    with _Knobs(intra_min_len=2500):
        with swmi.sw_db_load(mixed_db.residues, mixed_db.offsets, ALPHA) as h:
            with _Knobs(recompute_all=1, flag_cap=cap, route_len=route):
                _say(f"recompute-all through a list of {cap}, route {route}")
                single = h.search(qs[0], synth.BLOSUM62, 10, 2)
                batch = h.search_batch(qs, synth.BLOSUM62, 10, 2)
    want = [_oracle(q, mixed_db, synth.BLOSUM62, 10, 2) for q in qs]
    assert np.array_equal(single, want[0])
    for k in range(len(qs)):
        assert np.array_equal(batch[k], want[k]), k


@pytest.mark.parametrize("pairs", [0, 1])
def test_saturation_beyond_the_list(pairs):
    # SM(a, a) = 7: a^4681 and a^4682 saturate against the query a^4682 (32767, 32774);
    # with room for one entry the other is found by the overflow pass
    sm = np.array([[7, -3], [-3, 7]], dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(9))
    seqs = [np.zeros(4680, np.uint8), np.zeros(4681, np.uint8), np.zeros(4682, np.uint8),
            np.zeros(4682, np.uint8)]
    seqs += [rng.integers(0, 2, size=int(n)).astype(np.uint8) for n in rng.integers(3000, 4700, 60)]
    db = synth.db_from_seqs(seqs)
    qs = [np.zeros(4682, np.uint8), np.zeros(4681, np.uint8)]
    with _Knobs(flag_cap=1, route_len=1 << 30, query_pairs=pairs):
        with swmi.sw_db_load(db.residues, db.offsets, 2) as h:
            _say(f"saturation beyond a list of one, pairs={pairs}")
            got = h.search_batch(qs, sm, 10, 2)
    for k, q in enumerate(qs):
        want = _oracle(q, db, sm, 10, 2)
        assert np.array_equal(got[k], want), k
    assert list(got[0][:4]) == [32760, 32767, 32774, 32774]


def test_two_pair_items_beyond_the_list():
    # two pairs per wave in packed int16, both halves of some items saturating
    sm = np.array([[127, -3], [-3, 127]], dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(78))
    seqs = [np.zeros(n, np.uint8) for n in (257, 258, 259, 260, 1500, 1501)]
    seqs += [rng.integers(0, 2, size=int(n)).astype(np.uint8) for n in rng.integers(1, 1100, 30)]
    db = synth.db_from_seqs(seqs)
    q = np.zeros(1300, np.uint8)
    q[::97] = 1
    with _Knobs(flag_cap=1, route_len=1, intra_pairs=2):
        with swmi.sw_db_load(db.residues, db.offsets, 2) as h:
            _say("two-pair items beyond a list of one")
            got = h.search(q, sm, 10, 2)
    want = _oracle(q, db, sm, 10, 2)
    assert (want >= 32767).sum() >= 4
    assert np.array_equal(got, want)


def test_overflow_pass_in_a_captured_plan(mixed_db):
    import torch
    rng = np.random.Generator(np.random.PCG64(4242))
    qs = [synth.residues(rng, m) for m in (500, 260, 33)]
    want = np.stack([_oracle(q, mixed_db, synth.BLOSUM62, 10, 2) for q in qs])
    with _Knobs(intra_min_len=2500):
        with swmi.sw_db_load(mixed_db.residues, mixed_db.offsets, ALPHA) as h:
            out = torch.full((len(qs), mixed_db.n_seqs), -1, dtype=torch.int32, device="cuda")
            with _Knobs(recompute_all=1, flag_cap=3):
                plan = h.plan(qs, synth.BLOSUM62, 10, 2, out)
            try:
                for rep in range(3):
                    out.fill_(-1)
                    _say(f"plan replay {rep} with the overflow pass")
                    plan.launch()
                    torch.cuda.synchronize()
                    assert np.array_equal(out.cpu().numpy(), want), rep
                    # eager work between replays
                    assert np.array_equal(h.search(qs[1], synth.BLOSUM62, 10, 2), want[1])
            finally:
                plan.free()
