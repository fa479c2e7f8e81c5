"""Autotuner: binning and cache on the CPU; configurations agree on the GPU."""
from __future__ import annotations

import json

import numpy as np
import pytest

from paper_1702_07195_amd import autotune, synth


def test_bins_sorted_and_complete():
    qs = [np.zeros(n, np.uint8) for n in (5, 50, 7, 300, 1, 44, 44)]
    for width in (0, 1, 2, 3, 7, 100):
        b = autotune.bins(qs, width)
        flat = [k for x in b for k in x]
        assert sorted(flat) == list(range(len(qs)))
        lens = [len(qs[k]) for k in flat]
        assert lens == sorted(lens, reverse=True)
        if 0 < width < len(qs):
            assert all(len(x) <= width for x in b)


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv("SWMI_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    cache = {"k": {"config": autotune.Config(24, 8, 16).as_dict(), "timings": {}}}
    autotune._save_cache(cache)
    assert autotune._load_cache() == cache
    assert json.load(open(tmp_path / "c.json"))["k"]["config"]["bin_width"] == 16


@pytest.mark.gpu
def test_configurations_give_identical_scores(tmp_path, monkeypatch):
    import torch
    import oracle
    from paper_1702_07195_amd import swmi
    monkeypatch.setenv("SWMI_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    rng = np.random.Generator(np.random.PCG64(41))
    db = synth.db_from_lengths(rng, synth.lognormal_lengths(rng, 900, 150, 0.8, 1, 1200))
    qs = synth.batched_queries(7, 20, 600, seed=42)
    want = np.stack([oracle.search(q, db.residues, db.offsets, synth.BLOSUM62, 10, 2) for q in qs])
    with swmi.sw_db_load(db.residues, db.offsets, len(synth.ALPHABET)) as h:
        out = torch.zeros((len(qs), db.n_seqs), dtype=torch.int32, device="cuda")
        cands = [autotune.Config(t, w, b) for t, w, b in
                 ((16, 0, 0), (24, 8, 3), (40, 0, 2), (32, 12, 0))]
        for c in cands:
            print(f"config {c}", flush=True)
            out.fill_(-1)
            p = autotune.BinnedPlans(h, qs, synth.BLOSUM62, 10, 2, out, c)
            try:
                p.launch(torch.cuda.current_stream())
                torch.cuda.synchronize()
                p.gather()
            finally:
                p.free()
            assert np.array_equal(out.cpu().numpy(), want), c
        best, timings = autotune.tune(h, int(db.offsets[-1]), qs, synth.BLOSUM62, 10, 2, out,
                                      candidates=cands)
        assert best in cands and len(timings) == len(cands)
        again, _ = autotune.tune(h, int(db.offsets[-1]), qs, synth.BLOSUM62, 10, 2, out)
        assert again == best  # served from the cache
