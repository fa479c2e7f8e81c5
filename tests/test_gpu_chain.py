"""GPU parity of chained bands in the intra-task kernel.

A pair swept by a single wave may run its query bands back to back as one stream
(SW_KNOB_INTRA_CHAIN): lanes entering a new band clear their rows' H and E, and the band
boundary rows go through one linear buffer.  That needs n >= 192 residues (a bottom-row
entry is written before the lane below the band reads it), two or more bands, and a
buffer of nb * n + 128 entries within the wave's ring (twice the database's longest
sequence + 128, rounded up to 64); other pairs sweep band after band.  The databases
below put sequence lengths on both sides of each limit (191/192 residues, one band or
several, buffers that fit and that do not), single pairs in int32 and two-pair items
in packed int16, and every score must equal the oracle's and the band-after-band
sweep's.
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


@pytest.fixture(scope="module")
def edge_db():
    # longest sequence 1100: each wave's ring holds 2 * 1280 entries, so with 128-row
    # bands a 600-residue query (5 bands) chains pairs up to 486 residues and sweeps the
    # longer ones band after band
    rng = np.random.Generator(np.random.PCG64(6061))
    lengths = np.concatenate([[190, 191, 192, 193, 255, 256, 257, 486, 487, 1100, 1100, 0, 5],
                              rng.integers(150, 1100, 70)])
    return synth.db_from_lengths(rng, lengths)


@pytest.mark.parametrize("pairs", [0, 2])
@pytest.mark.parametrize("R,m", [(2, 129), (2, 250), (2, 600), (4, 700), (8, 1100),
                                 (16, 1500), (16, 2049)])
def test_chained_bands_equal_the_oracle(edge_db, R, m, pairs):
    rng = np.random.Generator(np.random.PCG64(7000 + m + R))
    q = synth.residues(rng, m)
    want = oracle.search(q, edge_db.residues, edge_db.offsets, synth.BLOSUM62, 10, 2)
    got = {}
    with swmi.sw_db_load(edge_db.residues, edge_db.offsets, ALPHA) as h:
        for chain in (1, 0):
            with _Knobs(route_len=1, intra_rows=R, intra_pairs=pairs, intra_chain=chain):
                _say(f"chained bands R={R} m={m} pairs={pairs} chain={chain}")
                got[chain] = h.search(q, synth.BLOSUM62, 10, 2)
    assert np.array_equal(got[1], want)
    assert np.array_equal(got[0], want)


def test_chained_two_pair_items_with_saturation():
    # SM(a, a) = 127 on a two-letter alphabet: a^258 scores 32766 (exact in int16),
    # a^259 and longer saturate and are recomputed in int32, in chained two-pair items
    # with partners of other lengths
    sm = np.array([[127, -3], [-3, 127]], dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(8080))
    seqs = [np.zeros(n, np.uint8) for n in (192, 257, 258, 259, 300, 700)]
    seqs += [rng.integers(0, 2, size=int(n)).astype(np.uint8) for n in rng.integers(192, 1100, 30)]
    db = synth.db_from_seqs(seqs)
    q = np.zeros(1300, np.uint8)
    q[::97] = 1
    want = oracle.search(q, db.residues, db.offsets, sm, 10, 2)
    assert want[2] < 32767 <= want[3]
    with swmi.sw_db_load(db.residues, db.offsets, 2) as h:
        for R in (2, 4):
            with _Knobs(route_len=1, intra_rows=R, intra_pairs=2, intra_chain=1):
                _say(f"chained two-pair items with saturation R={R}")
                assert np.array_equal(h.search(q, sm, 10, 2), want), R


def test_chained_bands_in_a_batch_and_a_captured_plan(edge_db):
    import torch
    rng = np.random.Generator(np.random.PCG64(9191))
    qs = [synth.residues(rng, m) for m in (700, 193, 1500, 60)]
    want = np.stack([oracle.search(q, edge_db.residues, edge_db.offsets, synth.BLOSUM62, 10, 2)
                     for q in qs])
    with swmi.sw_db_load(edge_db.residues, edge_db.offsets, ALPHA) as h:
        with _Knobs(route_len=1, intra_rows=4, intra_chain=1):
            _say("chained bands, batch")
            assert np.array_equal(h.search_batch(qs, synth.BLOSUM62, 10, 2), want)
            out = torch.full((len(qs), edge_db.n_seqs), -1, dtype=torch.int32, device="cuda")
            plan = h.plan(qs, synth.BLOSUM62, 10, 2, out)
        try:
            for rep in range(3):
                out.fill_(-1)
                _say(f"chained bands, plan replay {rep}")
                plan.launch()
                torch.cuda.synchronize()
                assert np.array_equal(out.cpu().numpy(), want), rep
        finally:
            plan.free()
