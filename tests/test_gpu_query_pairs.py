"""GPU parity of the two-query inter-task kernel (batched searches, SW_KNOB_QUERY_PAIRS).

Every score of a batched search must equal the oracle's, with the queries paired two
per lane (the default) and with pairing off; odd query counts, pairs of very different
lengths, empty queries, every compiled strip height and saturation in one half of a
pair are covered.
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


@pytest.fixture(scope="module")
def pdb():
    rng = np.random.Generator(np.random.PCG64(4242))
    lengths = synth.lognormal_lengths(rng, 400, 110, 0.8, 0, 700)
    lengths[:4] = [0, 1, 5, 0]
    return synth.db_from_lengths(rng, lengths)


@pytest.fixture(scope="module")
def phandle(pdb):
    _say(f"load pair-test db: {pdb.n_seqs} seqs, {pdb.offsets[-1]} residues")
    h = swmi.sw_db_load(pdb.residues, pdb.offsets, ALPHA)
    yield h
    h.free()


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


def _want(qs, db, sm, go, ge):
    return np.stack([oracle.search(q, db.residues, db.offsets, sm, go, ge) for q in qs])


def _queries(lens, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [synth.residues(rng, m) for m in lens]


# query lengths around strip boundaries (multiples of 8 .. 40), an empty query, and
# partners of very different lengths in the same pair
LENGTH_SETS = {
    "two": [97, 96],
    "odd3": [48, 300, 7],
    "ragged7": [0, 1, 8, 9, 40, 41, 333],
    "uneven": [600, 3, 250, 249, 24, 25],
}


@pytest.mark.parametrize("name", sorted(LENGTH_SETS))
@pytest.mark.parametrize("T", [8, 16, 24, 28, 32, 40])
def test_pairs_equal_oracle_at_every_strip_height(pdb, phandle, name, T):
    qs = _queries(LENGTH_SETS[name], seed=len(name) * 31 + T)
    want = _want(qs, pdb, synth.BLOSUM62, 10, 2)
    _say(f"pairs {name} T={T}")
    with _Knobs(strip_rows=T, route_len=1 << 30, query_pairs=1):
        got = phandle.search_batch(qs, synth.BLOSUM62, 10, 2)
    for k in range(len(qs)):
        assert np.array_equal(got[k], want[k]), (name, T, k, len(qs[k]))


@pytest.mark.parametrize("route", [0, 1 << 30])
@pytest.mark.parametrize("mat,go,ge", [("BLOSUM50", 11, 1), ("BLOSUM62", 10, 2),
                                        ("BLOSUM62", 0, 0), ("BLOSUM62", 16383, 0)])
def test_pairs_on_equal_pairs_off(pdb, phandle, route, mat, go, ge):
    qs = synth.batched_queries(9, 1, 500, seed=77)
    sm = synth.MATRICES[mat]
    _say(f"pairs on/off {mat} {go}/{ge} route={route}")
    with _Knobs(route_len=route, query_pairs=1):
        on = phandle.search_batch(qs, sm, go, ge)
    with _Knobs(route_len=route, query_pairs=0):
        off = phandle.search_batch(qs, sm, go, ge)
    assert np.array_equal(on, off)
    want = _want(qs, pdb, sm, go, ge)
    assert np.array_equal(on, want)


@pytest.mark.parametrize("recompute_all", [0, 1])
def test_saturation_in_one_half_of_a_pair(recompute_all):
    # SM(a, a) = 7: the query a^4682 saturates against a^4681 and a^4682 (scores 32767
    # and 32774) and must be recomputed in int32; its partner, a shorter query, never
    # saturates and keeps its int16 scores (unless every score is recomputed).
    sm = np.array([[7, -3], [-3, 7]], dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(19))
    seqs = [np.zeros(4680, np.uint8), np.zeros(4681, np.uint8), np.zeros(4682, np.uint8)]
    seqs += [rng.integers(0, 2, size=int(n)).astype(np.uint8) for n in rng.integers(3000, 4700, 70)]
    db = synth.db_from_seqs(seqs)
    qs = [np.zeros(4682, np.uint8), rng.integers(0, 2, size=4000).astype(np.uint8),
          np.zeros(4681, np.uint8)]
    want = _want(qs, db, sm, 10, 2)
    assert list(want[0][:3]) == [32760, 32767, 32774]
    assert list(want[2][:3]) == [32760, 32767, 32767]
    _say(f"pair saturation recompute_all={recompute_all}")
    with _Knobs(route_len=1 << 30, query_pairs=1, recompute_all=recompute_all):
        with swmi.sw_db_load(db.residues, db.offsets, 2) as h:
            got = h.search_batch(qs, sm, 10, 2)
    for k in range(len(qs)):
        assert np.array_equal(got[k], want[k]), k


def test_pairs_in_a_captured_plan(pdb, phandle):
    import torch
    qs = synth.batched_queries(5, 1, 400, seed=91)
    want = _want(qs, pdb, synth.BLOSUM62, 10, 2)
    out = torch.full((len(qs), pdb.n_seqs), -1, dtype=torch.int32, device="cuda")
    _say("pairs in a plan")
    with _Knobs(query_pairs=1):
        with phandle.plan(qs, synth.BLOSUM62, 10, 2, out) as plan:
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), want), "eager run"
            for rep in range(3):
                out.fill_(-1)
                torch.cuda.synchronize()
                plan.launch()
                torch.cuda.synchronize()
                assert np.array_equal(out.cpu().numpy(), want), f"replay {rep}"
                one = phandle.search(qs[rep], synth.BLOSUM62, 10, 2)
                assert np.array_equal(one, want[rep])


def test_pair_only_height_on_a_single_query(pdb, phandle):
    # 28 rows exist only in the pair kernel: a single-query search with that height forced
    # chooses its own height and stays exact
    rng = np.random.Generator(np.random.PCG64(28))
    q = synth.residues(rng, 210)
    _say("single query with strip rows 28")
    with _Knobs(strip_rows=28, route_len=1 << 30):
        got = phandle.search(q, synth.BLOSUM62, 10, 2)
    assert np.array_equal(got, oracle.search(q, pdb.residues, pdb.offsets, synth.BLOSUM62, 10, 2))


def test_two_widths_of_boundary_slots():
    # 64 queries against a database whose groups fill the device many times over: one
    # boundary slot per wave as wide as the widest group would pass the slot budget, so the
    # widest groups go to an eighth of the waves (full-width slots) and the others' slots
    # are as wide as the remaining groups.  Scores must equal those of one query per lane
    # (every score) and the oracle's (the widest sequences and a sample of the others).
    rng = np.random.Generator(np.random.PCG64(6464))
    lengths = synth.lognormal_lengths(rng, 60000, 200, 0.8, 10, 8000)
    db = synth.db_from_lengths(rng, lengths)
    qs = [synth.residues(rng, int(m)) for m in rng.integers(30, 121, size=64)]
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        _say("64 queries, two classes of boundary slots")
        got = h.search_batch(qs, synth.BLOSUM62, 10, 2)
        st = h.stats()
        with _Knobs(query_pairs=0):
            _say("the same batch, one query per lane")
            single = h.search_batch(qs, synth.BLOSUM62, 10, 2)
    assert st["query_pairs"] == 1 and st["big_waves"] > 0, st
    assert np.array_equal(got, single)
    order = np.argsort(lengths, kind="stable")
    idx = np.concatenate([order[-640:], rng.choice(order[:-640], 300, replace=False)])
    for k in range(0, len(qs), 7):
        want = oracle.search(qs[k], db.residues, db.offsets, synth.BLOSUM62, 10, 2, index=idx)
        assert np.array_equal(got[k][idx], want), k
