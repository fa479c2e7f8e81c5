"""GPU parity: scores from the HIP path (through the C ABI) equal the oracle's exactly.

Inputs are seeded synthetic databases and queries at sizes the oracle finishes in
seconds, spanning several groups of 64 sequences, several strips and bands, and ragged
tails.  Integer scores must match bit for bit.
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
def small_db():
    rng = np.random.Generator(np.random.PCG64(20250))
    lengths = synth.lognormal_lengths(rng, 700, 120, 0.9, 0, 900)
    lengths[:5] = [0, 1, 2, 3, 0]
    return synth.db_from_lengths(rng, lengths)


@pytest.fixture(scope="module")
def small_handle(small_db):
    _say(f"load small db: {small_db.n_seqs} seqs, {small_db.offsets[-1]} residues")
    h = swmi.sw_db_load(small_db.residues, small_db.offsets, ALPHA)
    yield h
    h.free()


def _oracle(q, db, sm, go, ge):
    return oracle.search(q, db.residues, db.offsets, sm, go, ge)


# Search-time routing of long groups: everything through the inter-task kernel, the
# automatic threshold, or everything through the intra-task kernel.
ROUTES = {"inter": 1 << 30, "auto": 0, "intra": 1}


@pytest.fixture(params=sorted(ROUTES))
def route(request):
    old = swmi.get_knob(swmi.SW_KNOB_ROUTE_LEN)
    swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, ROUTES[request.param])
    yield request.param
    swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, old)


@pytest.fixture
def inter_only():
    old = swmi.get_knob(swmi.SW_KNOB_ROUTE_LEN)
    swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, 1 << 30)
    yield
    swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, old)


@pytest.mark.parametrize("m", [1, 5, 31, 32, 33, 47, 48, 64, 65, 144, 200, 511, 1025, 2100])
def test_query_lengths_blosum62(small_db, small_handle, m, route):
    rng = np.random.Generator(np.random.PCG64(1000 + m))
    q = synth.residues(rng, m)
    _say(f"search m={m} route={route}")
    got = small_handle.search(q, synth.BLOSUM62, 10, 2)
    assert np.array_equal(got, _oracle(q, small_db, synth.BLOSUM62, 10, 2))


@pytest.mark.parametrize("mat,go,ge", [("BLOSUM50", 10, 2), ("BLOSUM62", 11, 1),
                                        ("BLOSUM50", 11, 1), ("BLOSUM62", 0, 0),
                                        ("BLOSUM62", 0, 5), ("BLOSUM62", 40, 0),
                                        ("BLOSUM62", 16383, 0)])
def test_matrices_and_gaps(small_db, small_handle, mat, go, ge, route):
    rng = np.random.Generator(np.random.PCG64(77))
    q = synth.residues(rng, 180)
    sm = synth.MATRICES[mat]
    _say(f"search {mat} {go}/{ge}")
    assert np.array_equal(small_handle.search(q, sm, go, ge), _oracle(q, small_db, sm, go, ge))


def test_asymmetric_small_alphabet():
    rng = np.random.Generator(np.random.PCG64(31337))
    alpha = 4
    lengths = synth.lognormal_lengths(rng, 200, 60, 0.8, 0, 300)
    seqs = [rng.integers(0, alpha, size=int(n)).astype(np.uint8) for n in lengths]
    db = synth.db_from_seqs(seqs)
    sm = synth.random_matrix(rng, alpha, -9, 12)
    q = rng.integers(0, alpha, size=97).astype(np.uint8)
    _say("search asymmetric alphabet 4")
    with swmi.sw_db_load(db.residues, db.offsets, alpha) as h:
        assert np.array_equal(h.search(q, sm, 3, 1), _oracle(q, db, sm, 3, 1))


@pytest.mark.parametrize("T", [8, 16, 24, 32, 40])
def test_strip_heights_agree(small_db, small_handle, T, inter_only):
    rng = np.random.Generator(np.random.PCG64(5))
    q = synth.residues(rng, 150)
    swmi.set_knob(swmi.SW_KNOB_STRIP_ROWS, T)
    try:
        _say(f"search strip rows T={T}")
        got = small_handle.search(q, synth.BLOSUM62, 10, 2)
    finally:
        swmi.set_knob(swmi.SW_KNOB_STRIP_ROWS, 0)
    assert np.array_equal(got, _oracle(q, small_db, synth.BLOSUM62, 10, 2))


def test_recompute_all_changes_nothing(small_db, small_handle, route):
    rng = np.random.Generator(np.random.PCG64(6))
    q = synth.residues(rng, 260)
    swmi.set_knob(swmi.SW_KNOB_RECOMPUTE_ALL, 1)
    try:
        _say("search recompute-all")
        got = small_handle.search(q, synth.BLOSUM62, 10, 2)
    finally:
        swmi.set_knob(swmi.SW_KNOB_RECOMPUTE_ALL, 0)
    assert np.array_equal(got, _oracle(q, small_db, synth.BLOSUM62, 10, 2))


@pytest.mark.parametrize("cut", [0, 50, 300])
def test_long_route_threshold(small_db, cut):
    rng = np.random.Generator(np.random.PCG64(8))
    q = synth.residues(rng, 1500)  # two intra-task bands
    old = swmi.get_knob(swmi.SW_KNOB_INTRA_MIN_LEN)
    swmi.set_knob(swmi.SW_KNOB_INTRA_MIN_LEN, cut)
    try:
        _say(f"load with intra threshold {cut}")
        with swmi.sw_db_load(small_db.residues, small_db.offsets, ALPHA) as h:
            got = h.search(q, synth.BLOSUM62, 10, 2)
    finally:
        swmi.set_knob(swmi.SW_KNOB_INTRA_MIN_LEN, old)
    assert np.array_equal(got, _oracle(q, small_db, synth.BLOSUM62, 10, 2))


def test_saturation_and_exact_recompute(route):
    # SM(a, a) = 7: a^4680 scores 32760 (exact in int16), a^4681 = 32767 and
    # a^4682 = 32774 saturate and must be recomputed exactly in int32; neighbours in the
    # same group keep their int16 scores.
    sm = np.array([[7, -3], [-3, 7]], dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(9))
    seqs = [np.zeros(4680, np.uint8), np.zeros(4681, np.uint8), np.zeros(4682, np.uint8)]
    seqs += [rng.integers(0, 2, size=int(n)).astype(np.uint8) for n in rng.integers(4000, 4700, 70)]
    db = synth.db_from_seqs(seqs)
    q = np.zeros(4682, np.uint8)
    _say("search saturation")
    with swmi.sw_db_load(db.residues, db.offsets, 2) as h:
        got = h.search(q, sm, 10, 2)
    want = _oracle(q, db, sm, 10, 2)
    assert list(want[:3]) == [32760, 32767, 32774]
    assert np.array_equal(got, want)


def test_empty_cases():
    _say("empty database")
    with swmi.sw_db_load(np.zeros(0, np.uint8), np.zeros(1, np.int64), ALPHA) as h:
        assert h.size() == 0
        assert h.search(synth.encode("ACDE"), synth.BLOSUM62, 10, 2).shape == (0,)
    db = synth.db_from_seqs([synth.encode("ACDEFG"), np.zeros(0, np.uint8), synth.encode("W")])
    _say("empty query / empty sequences")
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        assert list(h.search(np.zeros(0, np.uint8), synth.BLOSUM62, 10, 2)) == [0, 0, 0]
        got = h.search(synth.encode("CDEF"), synth.BLOSUM62, 10, 2)
        assert np.array_equal(got, _oracle(synth.encode("CDEF"), db, synth.BLOSUM62, 10, 2))


def test_empty_query_after_a_search_scores_zero():
    # An empty query scores 0 against every sequence, also against sequences that the
    # search routes to the intra-task kernel (groups longer than 64 residues on a small
    # database) or that the database keeps for it (longer than 8192), and also right
    # after a search that left other scores in the pooled buffers; alone, in a batch and
    # asynchronously.
    import torch
    rng = np.random.Generator(np.random.PCG64(97))
    lengths = np.concatenate([[10, 100, 500, 9000, 20, 70, 8500],
                              rng.integers(1, 300, 150)])
    db = synth.db_from_lengths(rng, lengths)
    q = synth.residues(rng, 200)
    empty = np.zeros(0, np.uint8)
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        _say("search, then an empty query")
        want = h.search(q, synth.BLOSUM62, 10, 2)
        assert want.max() > 0
        assert not h.search(empty, synth.BLOSUM62, 10, 2).any()
        _say("batch with an empty query")
        got = h.search_batch([q, empty, q[:50]], synth.BLOSUM62, 10, 2)
        assert np.array_equal(got[0], want) and not got[1].any()
        _say("async empty query into a buffer holding other scores")
        out = torch.full((db.n_seqs,), 5, dtype=torch.int32, device="cuda")
        h.search_async(empty, synth.BLOSUM62, 10, 2, out)
        torch.cuda.synchronize()
        assert not out.cpu().numpy().any()
    assert np.array_equal(want, _oracle(q, db, synth.BLOSUM62, 10, 2))
    assert np.array_equal(got[2], _oracle(q[:50], db, synth.BLOSUM62, 10, 2))


def test_device_buffers_are_checked_by_the_binding(small_db, small_handle):
    # a wrong score tensor is refused before the library could write out of bounds
    import torch
    q = synth.encode("ACDEFGH")
    for bad in (torch.zeros(small_db.n_seqs, dtype=torch.int64, device="cuda"),
                torch.zeros(small_db.n_seqs - 1, dtype=torch.int32, device="cuda"),
                torch.zeros(2 * small_db.n_seqs, dtype=torch.int32, device="cuda")[::2],
                torch.zeros(small_db.n_seqs, dtype=torch.int32)):
        with pytest.raises(ValueError):
            small_handle.search_async(q, synth.BLOSUM62, 10, 2, bad)
        with pytest.raises(ValueError):
            small_handle.topk(bad, 5)
    with pytest.raises(ValueError):
        small_handle.plan([q, q], synth.BLOSUM62, 10, 2,
                          torch.zeros(small_db.n_seqs, dtype=torch.int32, device="cuda"))


def test_bad_search_arguments(small_handle):
    with pytest.raises(swmi.SwError) as e:
        small_handle.search(np.array([0, 40], np.uint8), synth.BLOSUM62, 10, 2)
    assert e.value.code == swmi.SW_EINVAL
    bad = synth.BLOSUM62.copy()
    bad[0, 0] = 128
    with pytest.raises(swmi.SwError):
        small_handle.search(synth.encode("ACD"), bad, 10, 2)
    with pytest.raises(swmi.SwError):
        small_handle.search(synth.encode("ACD"), synth.BLOSUM62, -1, 2)
    with pytest.raises(swmi.SwError):
        small_handle.search(synth.encode("ACD"), synth.BLOSUM62, 16383, 1)


def test_batch_equals_separate(small_db, small_handle, route):
    qs = synth.batched_queries(6, 1, 400, seed=11)
    _say("batched search of 6 queries")
    got = small_handle.search_batch(qs, synth.BLOSUM62, 10, 2)
    for k, q in enumerate(qs):
        assert np.array_equal(got[k], _oracle(q, small_db, synth.BLOSUM62, 10, 2)), k


def test_async_on_torch_stream(small_db, small_handle):
    import torch
    rng = np.random.Generator(np.random.PCG64(12))
    q = synth.residues(rng, 222)
    out = torch.full((small_db.n_seqs,), -1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    _say("async search on a torch stream")
    small_handle.search_async(q, synth.BLOSUM62, 10, 2, out, stream)
    stream.synchronize()
    assert np.array_equal(out.cpu().numpy(), _oracle(q, small_db, synth.BLOSUM62, 10, 2))


def test_order_independence(small_db, small_handle):
    rng = np.random.Generator(np.random.PCG64(13))
    q = synth.residues(rng, 120)
    perm = rng.permutation(small_db.n_seqs)
    pdb = synth.db_from_seqs([small_db.seq(int(k)) for k in perm])
    base = small_handle.search(q, synth.BLOSUM62, 10, 2)
    _say("permuted database")
    with swmi.sw_db_load(pdb.residues, pdb.offsets, ALPHA) as h:
        assert np.array_equal(h.search(q, synth.BLOSUM62, 10, 2), base[perm])


def test_plan_graph_replays(small_db, small_handle, route):
    # A captured plan replayed several times, with eager searches and synchronisations
    # in between; every replay must equal the oracle (and the eager run).
    import torch
    qs = synth.batched_queries(5, 1, 700, seed=21)
    want = np.stack([_oracle(q, small_db, synth.BLOSUM62, 10, 2) for q in qs])
    out = torch.full((len(qs), small_db.n_seqs), -1, dtype=torch.int32, device="cuda")
    _say(f"plan create route={route}")
    with small_handle.plan(qs, synth.BLOSUM62, 10, 2, out) as plan:
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want), "eager run"
        stream = torch.cuda.Stream()
        for rep in range(3):
            out.fill_(-1)
            torch.cuda.synchronize()
            plan.launch(stream)
            stream.synchronize()
            assert np.array_equal(out.cpu().numpy(), want), f"replay {rep}"
            # eager work between replays
            other = small_handle.search(qs[rep], synth.BLOSUM50, 11, 1)
            assert np.array_equal(other, _oracle(qs[rep], small_db, synth.BLOSUM50, 11, 1))


def test_timing_per_kernel(small_db, small_handle):
    rng = np.random.Generator(np.random.PCG64(14))
    q = synth.residues(rng, 300)
    small_handle.timing_enable(True)
    small_handle.search(q, synth.BLOSUM62, 10, 2)
    small_handle.search(q, synth.BLOSUM62, 10, 2)
    n16, ms16 = small_handle.timing_read(swmi.SW_KERNEL_INTER16)
    nre, msre = small_handle.timing_read(swmi.SW_KERNEL_RECOMPUTE)
    small_handle.timing_enable(False)
    assert n16 in (0, 2) and nre == 2 and ms16 >= 0 and msre >= 0


def test_server_results_alone_equal_in_the_mix(small_db, small_handle):
    # Serving: each query's scores are identical when it is searched alone and when it
    # is submitted among others that arrive while earlier batches are on the GPU.
    import threading
    import time as _time
    qs = synth.served_queries(24, seed=31, median=120, lo=5, hi=600)
    alone = [small_handle.search(q, synth.BLOSUM62, 10, 2) for q in qs]
    _say("server mix")
    with swmi.SwServer(small_handle, synth.BLOSUM62, 10, 2, slots=3, max_batch=4) as sv:
        tickets = []
        for k, q in enumerate(qs):
            tickets.append(sv.submit(q))
            if k % 5 == 4:
                _time.sleep(0.002)  # let some batches start before the next arrivals
        results = [sv.wait(t) for t in tickets]
        st = sv.stats()
    for k, (scores, lat, qms) in enumerate(results):
        assert np.array_equal(scores, alone[k]), k
        assert lat >= qms >= 0
    assert st["launches"] >= 2
    for k in (0, 7, 23):
        assert np.array_equal(alone[k], _oracle(qs[k], small_db, synth.BLOSUM62, 10, 2))


def test_concurrent_searches_on_one_handle(small_db, small_handle):
    # Several host threads search the same database at once (single queries and
    # batches); the library's workspace pool holds two workspaces, so some calls wait
    # for one.  Every result equals the result of the same call made alone.
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.Generator(np.random.PCG64(41))
    qs = [synth.residues(rng, int(m)) for m in rng.integers(1, 400, 12)]
    batches = [qs[0:3], qs[3:5], qs[5:9]]
    alone_single = [small_handle.search(q, synth.BLOSUM62, 10, 2) for q in qs]
    alone_batch = [small_handle.search_batch(b, synth.BLOSUM62, 10, 2) for b in batches]

    def work(k):
        if k % 4 == 3:
            return ("b", k // 4, small_handle.search_batch(batches[k // 4], synth.BLOSUM62, 10, 2))
        return ("s", k, small_handle.search(qs[k], synth.BLOSUM62, 10, 2))

    _say("concurrent searches on one handle")
    with ThreadPoolExecutor(max_workers=6) as ex:
        results = list(ex.map(work, range(12)))
    for kind, k, got in results:
        want = alone_batch[k] if kind == "b" else alone_single[k]
        assert np.array_equal(got, want), (kind, k)
    assert np.array_equal(alone_single[5], _oracle(qs[5], small_db, synth.BLOSUM62, 10, 2))


def test_server_memory_admission(small_db, small_handle):
    # a budget smaller than one query's needs refuses it with SW_ENOMEM; others pass
    q = synth.served_queries(1, seed=32, median=100, lo=50, hi=150)[0]
    with swmi.SwServer(small_handle, synth.BLOSUM62, 10, 2, slots=1, max_batch=2,
                       mem_budget_bytes=1024) as sv:
        t = sv.submit(q)
        with pytest.raises(swmi.SwError) as e:
            sv.wait(t)
        assert e.value.code == swmi.SW_ENOMEM
        assert sv.stats()["refused"] == 1


def _expected_hits(scores, k):
    order = np.lexsort((np.arange(len(scores)), -scores.astype(np.int64)))
    return order[:k], scores[order[:k]]


@pytest.mark.parametrize("k", [1, 7, 100, 699, 700, 4096])
def test_topk_matches_oracle_order(small_db, small_handle, k):
    import torch
    rng = np.random.Generator(np.random.PCG64(51))
    q = synth.residues(rng, 90)
    want_scores = _oracle(q, small_db, synth.BLOSUM62, 10, 2)
    out = torch.zeros(small_db.n_seqs, dtype=torch.int32, device="cuda")
    small_handle.search_async(q, synth.BLOSUM62, 10, 2, out)
    _say(f"topk k={k}")
    idx, sc = small_handle.topk(out, k)
    wi, ws = _expected_hits(want_scores, min(k, small_db.n_seqs))
    assert np.array_equal(idx, wi) and np.array_equal(sc, ws)


def test_topk_ties_and_zero_scores():
    import torch
    seqs = [synth.encode("WWWW")] * 50 + [synth.encode("AAAA")] * 30 + [np.zeros(0, np.uint8)] * 20
    order = np.random.Generator(np.random.PCG64(52)).permutation(len(seqs))
    db = synth.db_from_seqs([seqs[i] for i in order])
    q = synth.encode("WWWWCC")
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        out = torch.zeros(db.n_seqs, dtype=torch.int32, device="cuda")
        h.search_async(q, synth.BLOSUM62, 10, 2, out)
        for k in (1, 49, 50, 51, 85, 100, 200):
            idx, sc = h.topk(out, k)
            wi, ws = _expected_hits(out.cpu().numpy(), min(k, db.n_seqs))
            assert np.array_equal(idx, wi) and np.array_equal(sc, ws), k
        with pytest.raises(swmi.SwError):
            h.topk(out, 4097)


def test_search_of_fasta_database(tmp_path):
    from paper_1702_07195_amd import fasta
    rng = np.random.Generator(np.random.PCG64(62))
    db = synth.db_from_lengths(rng, synth.lognormal_lengths(rng, 300, 150, 0.8, 1, 900))
    fasta.write_fasta(str(tmp_path / "d.fa"), [f"s{k}" for k in range(db.n_seqs)], db)
    _, db2 = fasta.read_fasta(str(tmp_path / "d.fa"))
    fasta.save_binary(str(tmp_path / "d.swdb"), db2)
    db3, alpha = fasta.load_binary(str(tmp_path / "d.swdb"))
    q = synth.residues(rng, 222)
    with swmi.sw_db_load(db3.residues, db3.offsets, alpha) as h:
        got = h.search(q, synth.BLOSUM62, 10, 2)
    assert np.array_equal(got, _oracle(q, db, synth.BLOSUM62, 10, 2))


@pytest.mark.parametrize("waves", [0, 4, 8])
@pytest.mark.parametrize("m,cap", [(9000, 0), (17000, 0), (17000, 2), (17000, 1)])
def test_split_pairs_across_workgroups(m, cap, waves):
    # Queries with more query bands than a workgroup has waves: wide pairs are split
    # into segments on different workgroups that hand the boundary row over through
    # global memory (cap: most segments per pair, 0 = automatic, 1 = none; waves per
    # workgroup 4, 8 or automatic); every sequence is routed to the intra-task kernel.
    rng = np.random.Generator(np.random.PCG64(70 + m))
    lengths = np.concatenate([rng.integers(1200, 3000, 6), rng.integers(1, 900, 40)])
    db = synth.db_from_lengths(rng, lengths)
    q = synth.residues(rng, m)
    knobs = (swmi.SW_KNOB_ROUTE_LEN, swmi.SW_KNOB_MAX_SEGMENTS, swmi.SW_KNOB_MAIN_WAVES)
    old = [swmi.get_knob(k) for k in knobs]
    for k, v in zip(knobs, (1, cap, waves)):
        swmi.set_knob(k, v)
    try:
        _say(f"split pairs m={m} cap={cap} waves={waves}")
        with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
            got = h.search(q, synth.BLOSUM62, 10, 2)
    finally:
        for k, v in zip(knobs, old):
            swmi.set_knob(k, v)
    assert np.array_equal(got, _oracle(q, db, synth.BLOSUM62, 10, 2))


@pytest.mark.parametrize("crit_rows", [0, 4, 8])
def test_critical_pairs(crit_rows):
    # 2,000 ordinary sequences and 10 of 15,000-30,000 residues against a 5,478-residue
    # query: the long pairs set the critical path and go to the critical-pair launch, in
    # bands of 256 or 512 rows (4 or 8 rows per lane, segments of four bands on
    # workgroups of their own), next to the main intra-task launch at 16 rows per lane.
    rng = np.random.Generator(np.random.PCG64(5478))
    lengths = np.concatenate([synth.lognormal_lengths(rng, 2000, 300, 0.8, 10, 8000),
                              rng.integers(15000, 30000, 10)])
    db = synth.db_from_lengths(rng, lengths)
    q = synth.residues(rng, 5478)
    old = swmi.get_knob(swmi.SW_KNOB_CRIT_ROWS)
    swmi.set_knob(swmi.SW_KNOB_CRIT_ROWS, crit_rows)
    try:
        _say(f"critical pairs, rows per lane {crit_rows}")
        with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
            got = h.search(q, synth.BLOSUM62, 10, 2)
            st = h.stats()
    finally:
        swmi.set_knob(swmi.SW_KNOB_CRIT_ROWS, old)
    assert st["cells_crit"] > 0 and st["intra_rows"] == 16
    idx = np.concatenate([np.arange(2000, 2010), rng.choice(2000, 200, replace=False)])
    want = oracle.search(q, db.residues, db.offsets, synth.BLOSUM62, 10, 2, index=idx)
    assert np.array_equal(got[idx], want)


@pytest.mark.parametrize("share,prio", [(0, 0), (10, 1), (100, 1)])
def test_critical_share_and_wave_priority(share, prio):
    # the database of test_critical_pairs under other shares of the search time above
    # which a split long pair goes to the critical-pair launch, with wave priorities on
    # or off: scores must not change
    rng = np.random.Generator(np.random.PCG64(5478))
    lengths = np.concatenate([synth.lognormal_lengths(rng, 2000, 300, 0.8, 10, 8000),
                              rng.integers(15000, 30000, 10)])
    db = synth.db_from_lengths(rng, lengths)
    q = synth.residues(rng, 5478)
    knobs = (swmi.SW_KNOB_CRIT_SHARE, swmi.SW_KNOB_INTRA_PRIO)
    old = [swmi.get_knob(k) for k in knobs]
    cells = {}
    try:
        with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
            for s_, p_ in ((0, 1), (share, prio)):
                swmi.set_knob(swmi.SW_KNOB_CRIT_SHARE, s_)
                swmi.set_knob(swmi.SW_KNOB_INTRA_PRIO, p_)
                _say(f"critical share {s_}, intra priority {p_}")
                got = h.search(q, synth.BLOSUM62, 10, 2)
                cells[(s_, p_)] = h.stats()["cells_crit"]
    finally:
        for k, v in zip(knobs, old):
            swmi.set_knob(k, v)
    if share == 10:
        assert cells[(10, 1)] >= cells[(0, 1)]
    idx = np.concatenate([np.arange(2000, 2010), rng.choice(2000, 200, replace=False)])
    want = oracle.search(q, db.residues, db.offsets, synth.BLOSUM62, 10, 2, index=idx)
    assert np.array_equal(got[idx], want)


@pytest.fixture(scope="module")
def mixed_db():
    # lengths from empty to 3000 (narrow pairs below 1152, wide pairs above)
    rng = np.random.Generator(np.random.PCG64(4242))
    lengths = np.concatenate([rng.integers(0, 1152, 90), rng.integers(1152, 3000, 12)])
    return synth.db_from_lengths(rng, lengths)


@pytest.mark.parametrize("waves", [4, 8])
@pytest.mark.parametrize("R", [2, 4, 8, 16])
@pytest.mark.parametrize("m", [70, 300, 1500, 3000])
def test_intra_rows_per_lane(mixed_db, R, m, waves):
    # The intra-task kernel with bands of 64R rows (R query rows per lane) on workgroups
    # of 4 or 8 waves, every sequence routed to it; with small databases the longest
    # pairs are also split.
    rng = np.random.Generator(np.random.PCG64(900 + m))
    q = synth.residues(rng, m)
    knobs = (swmi.SW_KNOB_ROUTE_LEN, swmi.SW_KNOB_INTRA_ROWS, swmi.SW_KNOB_MAIN_WAVES)
    old = [swmi.get_knob(k) for k in knobs]
    for k, v in zip(knobs, (1, R, waves)):
        swmi.set_knob(k, v)
    try:
        _say(f"intra rows per lane R={R} m={m} waves={waves}")
        with swmi.sw_db_load(mixed_db.residues, mixed_db.offsets, ALPHA) as h:
            got = h.search(q, synth.BLOSUM62, 10, 2)
    finally:
        for k, v in zip(knobs, old):
            swmi.set_knob(k, v)
    assert np.array_equal(got, _oracle(q, mixed_db, synth.BLOSUM62, 10, 2))


def test_automatic_rows_with_very_long_sequences():
    # Sequences longer than the inter-task limit next to ordinary ones: the host picks the
    # rows per lane from throughput and the longest pair's path (few bands of 4 rows per
    # lane for the mid-length queries, 16 for the longest), splits long pairs across
    # workgroups as it sees fit, and every score still equals the oracle's, one query at
    # a time and in one batch.
    rng = np.random.Generator(np.random.PCG64(2718))
    lengths = np.concatenate([synth.lognormal_lengths(rng, 400, 300, 0.8, 10, 3000),
                              rng.integers(9000, 20001, 10)])
    db = synth.db_from_lengths(rng, lengths)
    qs = [synth.residues(rng, m) for m in (300, 1000, 2005, 5478)]
    want = [_oracle(q, db, synth.BLOSUM62, 10, 2) for q in qs]
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        for q, w in zip(qs, want):
            _say(f"automatic rows per lane, m={len(q)}")
            assert np.array_equal(h.search(q, synth.BLOSUM62, 10, 2), w), len(q)
        _say("automatic rows per lane, batch")
        assert np.array_equal(h.search_batch(qs, synth.BLOSUM62, 10, 2), np.stack(want))


@pytest.mark.parametrize("R", [0, 4, 16])
def test_paired_intra_items_with_saturation(R):
    # Two pairs per wave in packed int16 (wide and narrow items, every unsplit pair
    # paired): halves whose maximum reaches 32767 are recomputed in int32, the other half
    # of the same item keeps its int16 score.  SM(a, a) = 127: a^258 scores 32766 (exact),
    # a^259 32893 (saturates).
    sm = np.array([[127, -3], [-3, 127]], dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(77 + R))
    seqs = [np.zeros(257, np.uint8), np.zeros(258, np.uint8), np.zeros(259, np.uint8),
            np.zeros(1500, np.uint8)]
    seqs += [rng.integers(0, 2, size=int(n)).astype(np.uint8) for n in rng.integers(1, 1100, 41)]
    seqs += [rng.integers(0, 2, size=int(n)).astype(np.uint8) for n in rng.integers(1200, 2600, 9)]
    db = synth.db_from_seqs(seqs)
    q = np.zeros(1300, np.uint8)
    q[::97] = 1
    old = [swmi.get_knob(k) for k in (swmi.SW_KNOB_ROUTE_LEN, swmi.SW_KNOB_INTRA_PAIRS,
                                      swmi.SW_KNOB_INTRA_ROWS)]
    swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, 1)
    swmi.set_knob(swmi.SW_KNOB_INTRA_PAIRS, 2)
    swmi.set_knob(swmi.SW_KNOB_INTRA_ROWS, R)
    try:
        _say(f"paired intra items R={R}")
        with swmi.sw_db_load(db.residues, db.offsets, 2) as h:
            got = h.search(q, sm, 10, 2)
    finally:
        for k, v in zip((swmi.SW_KNOB_ROUTE_LEN, swmi.SW_KNOB_INTRA_PAIRS,
                         swmi.SW_KNOB_INTRA_ROWS), old):
            swmi.set_knob(k, v)
    want = _oracle(q, db, sm, 10, 2)
    assert want[1] < 32767 <= want[2]
    assert np.array_equal(got, want)


@pytest.mark.parametrize("m", [200, 2100])
def test_paired_intra_items_blosum(small_db, small_handle, m):
    # every unsplit intra-task pair paired, on the small database (empty sequences
    # included, an odd number of items per kind)
    rng = np.random.Generator(np.random.PCG64(5000 + m))
    q = synth.residues(rng, m)
    old = (swmi.get_knob(swmi.SW_KNOB_ROUTE_LEN), swmi.get_knob(swmi.SW_KNOB_INTRA_PAIRS))
    swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, 1)
    swmi.set_knob(swmi.SW_KNOB_INTRA_PAIRS, 2)
    try:
        _say(f"paired intra items m={m}")
        got = small_handle.search(q, synth.BLOSUM62, 10, 2)
    finally:
        swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, old[0])
        swmi.set_knob(swmi.SW_KNOB_INTRA_PAIRS, old[1])
    assert np.array_equal(got, _oracle(q, small_db, synth.BLOSUM62, 10, 2))


@pytest.mark.parametrize("case", range(12))
def test_random_configurations(case):
    # Seeded random configurations: alphabet, asymmetric matrix (entries up to the
    # +-127 bound), gap penalties, query length and database length law, with every
    # routing and pairing setting drawn at random; scores must equal the oracle's.
    rng = np.random.Generator(np.random.PCG64(31337 + case))
    alpha = int(rng.integers(2, 25))
    bound = int(rng.choice([3, 10, 127]))
    sm = synth.random_matrix(rng, alpha, -bound, bound)
    go, ge = int(rng.integers(0, 20)), int(rng.integers(0, 6))
    m = int(rng.choice([1, 7, 63, 300, 1100, 2500]))
    n_seqs = int(rng.integers(50, 400))
    lengths = synth.lognormal_lengths(rng, n_seqs, float(rng.choice([30, 150, 600])), 0.9, 0,
                                      3000)
    residues = rng.integers(0, alpha, size=int(lengths.sum()), dtype=np.uint8)
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    db = synth.SeqDB(residues, offsets)
    q = rng.integers(0, alpha, size=m, dtype=np.uint8)
    knobs = {swmi.SW_KNOB_ROUTE_LEN: int(rng.choice([0, 1, 1 << 30])),
             swmi.SW_KNOB_INTRA_PAIRS: int(rng.integers(0, 3)),
             swmi.SW_KNOB_INTRA_ROWS: int(rng.choice([0, 4, 8, 16])),
             swmi.SW_KNOB_STRIP_ROWS: int(rng.choice([0, 8, 16, 24, 32, 40]))}
    old = {k: swmi.get_knob(k) for k in knobs}
    try:
        for k, v in knobs.items():
            swmi.set_knob(k, v)
        _say(f"random case {case}: A={alpha} |SM|<={bound} gaps {go}/{ge} m={m} "
             f"n={n_seqs} knobs={list(knobs.values())}")
        with swmi.sw_db_load(db.residues, db.offsets, alpha) as h:
            got = h.search(q, sm, go, ge)
    finally:
        for k, v in old.items():
            swmi.set_knob(k, v)
    want = oracle.search(q, db.residues, db.offsets, sm, go, ge)
    assert np.array_equal(got, want)


def test_segment_wait_that_gives_up_fails_the_search():
    # A spin limit of one poll makes the waits between the segments of split pairs give
    # up: every kernel still runs to its end, the blocking search reports SW_EDEVICE,
    # and the next search (default limit) is exact again.
    rng = np.random.Generator(np.random.PCG64(88))
    lengths = np.concatenate([rng.integers(2000, 3000, 8), rng.integers(1, 900, 20)])
    db = synth.db_from_lengths(rng, lengths)
    q = synth.residues(rng, 17000)
    knobs = (swmi.SW_KNOB_ROUTE_LEN, swmi.SW_KNOB_SPIN_LIMIT, swmi.SW_KNOB_INTRA_PAIRS)
    old = [swmi.get_knob(k) for k in knobs]
    try:
        swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, 1)
        swmi.set_knob(swmi.SW_KNOB_INTRA_PAIRS, 0)
        with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
            swmi.set_knob(swmi.SW_KNOB_SPIN_LIMIT, 1)
            _say("search with a one-poll segment wait")
            out = np.full(db.n_seqs, -7, dtype=np.int32)
            qq = np.ascontiguousarray(q, dtype=np.uint8)
            sm = np.ascontiguousarray(synth.BLOSUM62, dtype=np.int32)
            rc = swmi.lib().sw_search(h.handle, qq.ctypes.data_as(swmi._u8p), len(qq),
                                      sm.ctypes.data_as(swmi._i32p), 10, 2,
                                      out.ctypes.data_as(swmi._i32p))
            assert rc == swmi.SW_EDEVICE
            assert (out == -7).all()  # a failed search leaves the output untouched
            swmi.set_knob(swmi.SW_KNOB_SPIN_LIMIT, 0)
            _say("search with the default limit")
            got = h.search(q, synth.BLOSUM62, 10, 2)
    finally:
        for k, v in zip(knobs, old):
            swmi.set_knob(k, v)
    assert np.array_equal(got, _oracle(q, db, synth.BLOSUM62, 10, 2))


def test_maximum_query_length():
    # The longest query the boundary accepts (2^24 residues) against a few short
    # sequences, through both kernels (1.1 GB of inter-task profile, 16,384 intra-task
    # bands split across workgroups); one residue more is rejected.
    rng = np.random.Generator(np.random.PCG64(2024))
    m = swmi.SW_MAX_QUERY_LEN
    q = synth.residues(rng, m)
    db = synth.db_from_seqs([synth.residues(rng, n) for n in (1, 7, 40)])
    want = oracle.search(q, db.residues, db.offsets, synth.BLOSUM62, 10, 2)
    old = swmi.get_knob(swmi.SW_KNOB_ROUTE_LEN)
    try:
        with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
            for route in (1 << 30, 1):
                swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, route)
                _say(f"maximum query length, route {route}")
                assert np.array_equal(h.search(q, synth.BLOSUM62, 10, 2), want), route
            with pytest.raises(swmi.SwError) as e:
                h.search(np.zeros(m + 1, np.uint8), synth.BLOSUM62, 10, 2)
            assert e.value.code == swmi.SW_EINVAL
    finally:
        swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, old)


@pytest.mark.parametrize("route", [0, 1])
def test_largest_alphabet(route):
    # 31 codes (the most the boundary accepts; code 31 is the padding code)
    rng = np.random.Generator(np.random.PCG64(3131 + route))
    sm = synth.random_matrix(rng, 31, -12, 12)
    lengths = synth.lognormal_lengths(rng, 300, 200, 0.9, 0, 2500)
    residues = rng.integers(0, 31, size=int(lengths.sum()), dtype=np.uint8)
    db = synth.SeqDB(residues, np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64))
    q = rng.integers(0, 31, size=700, dtype=np.uint8)
    old = swmi.get_knob(swmi.SW_KNOB_ROUTE_LEN)
    try:
        swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, route)
        with swmi.sw_db_load(db.residues, db.offsets, 31) as h:
            _say(f"alphabet 31, route {route}")
            got = h.search(q, sm, 7, 3)
    finally:
        swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, old)
    assert np.array_equal(got, oracle.search(q, db.residues, db.offsets, sm, 7, 3))


@pytest.mark.parametrize("pairs", [1, 2])
def test_split_two_pair_items(pairs):
    # Long sequences split across workgroups, two per workgroup in packed int16 (pairing
    # of split pairs: automatic when throughput-bound, or forced), their segments chained
    # through packed boundary rows and packed maxima; the oracle decides.
    rng = np.random.Generator(np.random.PCG64(606 + pairs))
    lengths = np.concatenate([rng.integers(9000, 12000, 12), rng.integers(1, 400, 100)])
    db = synth.db_from_lengths(rng, lengths)
    q = synth.residues(rng, 5000)
    old = swmi.get_knob(swmi.SW_KNOB_INTRA_PAIRS)
    swmi.set_knob(swmi.SW_KNOB_INTRA_PAIRS, pairs)
    try:
        with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
            _say(f"split two-pair items, pairs knob {pairs}")
            got = h.search(q, synth.BLOSUM62, 10, 2)
            st = h.stats()
    finally:
        swmi.set_knob(swmi.SW_KNOB_INTRA_PAIRS, old)
    if pairs == 2:
        assert st["cells_intra16"] > 0
    assert np.array_equal(got, _oracle(q, db, synth.BLOSUM62, 10, 2))


def test_split_two_pair_items_with_saturation():
    # SM(a, a) = 7, every pair routed to the intra-task kernel, every pair paired: the
    # split items pair a^4681 with a^4682 (and a^4680 with its neighbour); the saturated
    # halves (32767, 32774 against the query a^4700) are recomputed in int32, the others
    # keep their int16 scores.
    sm = np.array([[7, -3], [-3, 7]], dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(707))
    seqs = [np.zeros(n, np.uint8) for n in (4680, 4681, 4682)]
    seqs += [rng.integers(0, 2, size=int(n)).astype(np.uint8) for n in rng.integers(4600, 4700, 9)]
    db = synth.db_from_seqs(seqs)
    q = np.zeros(4700, np.uint8)
    knobs = (swmi.SW_KNOB_ROUTE_LEN, swmi.SW_KNOB_INTRA_PAIRS)
    old = [swmi.get_knob(k) for k in knobs]
    swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, 1)
    swmi.set_knob(swmi.SW_KNOB_INTRA_PAIRS, 2)
    try:
        with swmi.sw_db_load(db.residues, db.offsets, 2) as h:
            _say("split two-pair items with saturation")
            got = h.search(q, sm, 10, 2)
    finally:
        for k, v in zip(knobs, old):
            swmi.set_knob(k, v)
    want = _oracle(q, db, sm, 10, 2)
    assert list(want[:3]) == [32760, 32767, 32774]
    assert np.array_equal(got, want)
