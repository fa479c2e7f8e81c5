"""FASTA input and a binary database format (the paper converts FASTA to a binary file
once so that later runs load faster; Section 4, pre-processing stage).

Residue letters map to the codes of ``synth.ALPHABET`` (BLOSUM order); lower case is
accepted, and letters outside the alphabet (U, O, J, ...) map to X.

Binary format (little endian):  8-byte magic ``b"SWDB\\x01\\0\\0\\0"``, int64 n_seqs, int64
n_residues, int64 alphabet, int64 offsets[n_seqs + 1], uint8 residues[n_residues].
``load_binary`` memory-maps the two arrays, so a large database is not copied until it
is uploaded by ``sw_db_load``.
"""
from __future__ import annotations

import os

import numpy as np

from .synth import ALPHABET, CODE, SeqDB

MAGIC = b"SWDB\x01\x00\x00\x00"

_LUT = np.full(256, CODE["X"], dtype=np.uint8)
for _c, _v in CODE.items():
    _LUT[ord(_c)] = _v
    _LUT[ord(_c.lower())] = _v


def encode_bytes(text: bytes) -> np.ndarray:
    """Residue letters (bytes, whitespace removed) -> codes."""
    return _LUT[np.frombuffer(text, dtype=np.uint8)]


def read_fasta(path: str):
    """(names, SeqDB) of a FASTA file."""
    names, chunks, lengths = [], [], []
    cur = []
    with open(path, "rb") as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            if line.startswith(b">"):
                if names:
                    seq = b"".join(cur)
                    chunks.append(seq)
                    lengths.append(len(seq))
                names.append(line[1:].decode("utf-8", "replace"))
                cur = []
            else:
                cur.append(line)
    if names:
        seq = b"".join(cur)
        chunks.append(seq)
        lengths.append(len(seq))
    offsets = np.zeros(len(names) + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    residues = encode_bytes(b"".join(chunks)) if chunks else np.zeros(0, np.uint8)
    return names, SeqDB(residues, offsets)


def write_fasta(path: str, names, db: SeqDB, width: int = 60):
    letters = np.frombuffer(ALPHABET.encode(), dtype=np.uint8)
    with open(path, "wb") as f:
        for k, name in enumerate(names):
            f.write(b">" + name.encode() + b"\n")
            s = letters[db.seq(k)].tobytes()
            for i in range(0, len(s), width):
                f.write(s[i:i + width] + b"\n")


def save_binary(path: str, db: SeqDB, alphabet: int = len(ALPHABET)):
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        f.write(MAGIC)
        np.array([db.n_seqs, int(db.offsets[-1]), alphabet], dtype="<i8").tofile(f)
        np.ascontiguousarray(db.offsets, dtype="<i8").tofile(f)
        np.ascontiguousarray(db.residues, dtype=np.uint8).tofile(f)
    os.replace(tmp, path)


def load_binary(path: str):
    """(SeqDB, alphabet) of a binary database, with memory-mapped arrays."""
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError(f"{path}: not a binary sequence database")
        n, nres, alphabet = (int(x) for x in np.fromfile(f, dtype="<i8", count=3))
    head = 8 + 3 * 8
    offsets = np.memmap(path, dtype="<i8", mode="r", offset=head, shape=(n + 1,))
    residues = np.memmap(path, dtype=np.uint8, mode="r", offset=head + 8 * (n + 1),
                         shape=(nres,))
    if offsets[0] != 0 or offsets[-1] != nres:
        raise ValueError(f"{path}: inconsistent offsets")
    return SeqDB(residues, offsets), alphabet
