"""FASTA reader and binary database format (host side)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1702_07195_amd import fasta, synth


def test_fasta_round_trip_and_binary(tmp_path):
    rng = np.random.Generator(np.random.PCG64(61))
    db = synth.db_from_lengths(rng, synth.lognormal_lengths(rng, 137, 80, 0.9, 0, 400))
    names = [f"seq{k} synthetic" for k in range(db.n_seqs)]
    fa = tmp_path / "db.fa"
    fasta.write_fasta(str(fa), names, db, width=37)
    names2, db2 = fasta.read_fasta(str(fa))
    assert names2 == names
    assert np.array_equal(db2.offsets, db.offsets)
    assert np.array_equal(db2.residues, db.residues)
    b = tmp_path / "db.swdb"
    fasta.save_binary(str(b), db2)
    db3, alpha = fasta.load_binary(str(b))
    assert alpha == len(synth.ALPHABET)
    assert np.array_equal(np.asarray(db3.offsets), db.offsets)
    assert np.array_equal(np.asarray(db3.residues), db.residues)


def test_fasta_letters(tmp_path):
    fa = tmp_path / "x.fa"
    fa.write_text(">a\nACDEfghU\nw\n\n>empty\n>b desc\n*BZ\n")
    names, db = fasta.read_fasta(str(fa))
    assert names == ["a", "empty", "b desc"]
    assert synth.decode(db.seq(0)) == "ACDEFGHXW"
    assert db.lengths.tolist() == [9, 0, 3]
    assert synth.decode(db.seq(2)) == "*BZ"


def test_binary_rejects_garbage(tmp_path):
    p = tmp_path / "bad"
    p.write_bytes(b"NOTADB" + b"\0" * 64)
    with pytest.raises(ValueError):
        fasta.load_binary(str(p))
