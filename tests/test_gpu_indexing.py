"""Bit-exact checks of the default pass's own lookups and indexing, read back
through the C ABI (ara_debug_read):

* the fold's o(E) for every catalogue event equals the oracle's
  occurrence_catalogue bit for bit (Algorithm 3's lookup step, the per-ELT
  terms, the sum over ELTs in layer order and the occurrence terms, applied
  once per catalogue event);
* the compact array is exactly the nonzero o(E) in catalogue order, and the
  part images' bitmap words and ranks are those of the oracle's o(E);
* the 16-bit stream copy is the YET re-laid out: for every part and group of
  trials, each trial's events of that part in time order as part-relative
  IDs, groups padded to 16 bytes with 0xFFFF, and the group starts and trial
  ends that the pass reads.

Expected layouts are built here from the YET with NumPy indexing only (no
arithmetic of the method); expected o(E) comes from the oracle.
"""

import numpy as np
import pytest

import oracle
from workloads import Layer, make_config, make_elt_pool, make_tiny_yet, make_yet

pytestmark = pytest.mark.gpu

IMG_BYTES = 37120


@pytest.fixture(scope="module")
def ara():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1606_04473_amd import ara as mod
    mod.lib()
    return mod


def _check_fold(ara, tables, pool, layer, yet):
    spec = ara.LayerSpec.from_layer(layer, pool, yet.n_trials)
    o = ara.debug_read(tables, ara.DEBUG_OCCURRENCE, spec)
    _, o_ref = oracle.occurrence_catalogue(pool, layer)
    assert o.shape == o_ref.shape
    assert np.array_equal(o.view(np.uint64), o_ref.view(np.uint64))
    nz = np.flatnonzero(o_ref != 0.0)
    comp = ara.debug_read(tables, ara.DEBUG_COMPACT, spec)
    assert np.array_equal(comp.view(np.uint64), o_ref[nz].view(np.uint64))
    # part images: bitmap bits, ranks inside superblocks, superblock ranks
    img = ara.debug_read(tables, ara.DEBUG_IMAGES, spec)
    P = img.shape[0] // IMG_BYTES
    C = o_ref.shape[0]
    flags = np.zeros(P << 18, dtype=np.uint8)
    flags[:C] = o_ref != 0.0
    for p in range(P):
        rec = img[p * IMG_BYTES:(p + 1) * IMG_BYTES]
        words = rec[:32768].view(np.uint64)
        r16 = rec[32768:32768 + 4096].view(np.uint16)
        b32 = rec[32768 + 4096:].view(np.uint32)
        f = flags[p << 18:(p + 1) << 18]
        want_words = np.packbits(f.reshape(-1, 64)[:, ::-1], axis=1).view(">u8").ravel().astype(np.uint64)
        assert np.array_equal(words, want_words), p
        per128 = f.reshape(-1, 128).sum(axis=1, dtype=np.int64)
        within = per128.reshape(-1, 32)
        want_r16 = (np.cumsum(within, axis=1) - within).ravel()
        assert np.array_equal(r16.astype(np.int64), want_r16), p
        before = int(flags[:p << 18].sum(dtype=np.int64))
        per_sb = f.reshape(-1, 4096).sum(axis=1, dtype=np.int64)
        want_b32 = before + np.cumsum(per_sb) - per_sb
        assert np.array_equal(b32.astype(np.int64), want_b32), p
    return o


def test_fold_outputs_bit_exact(ara):
    """config0, a dense-ELT catalogue of several parts and a layer whose ELT
    order is reversed: o(E), the compact values and the part images."""
    w = make_config("config0")
    tables = ara.create_tables(w.yet.offsets, w.yet.ids, w.pool.losses)
    _check_fold(ara, tables, w.pool, w.layers[0], w.yet)
    tables.close()
    C = 600_000
    yet = make_yet(50, 20.0, C, seed=181)
    pool = make_elt_pool(12, C, 300_000, seed=182)
    tables = ara.create_tables(yet.offsets, yet.ids, pool.losses)
    idx = np.array([11, 3, 7, 0, 9, 1, 5, 10, 2, 6], dtype=np.int32)
    for lay in (Layer(idx, 2500.0, 2.0e6, 1.2e8, 2.0e7), Layer(idx[::-1].copy(), 0.0, np.inf, 0.0, np.inf)):
        _check_fold(ara, tables, pool, lay, yet)
    tables.close()


def test_fold_outputs_bit_exact_config1(ara):
    """The 1M-trial workload's layer: o(E) of all 2M catalogue events, the
    compact values and the images, bit for bit."""
    w = make_config("config1", n_prefix=1000)
    tables = ara.create_tables(w.yet.offsets, w.yet.ids, w.pool.losses)
    o = _check_fold(ara, tables, w.pool, w.layers[0], w.yet)
    assert 0.10 < np.mean(o != 0.0) < 0.20
    tables.close()


def _expected_stream(yet, G):
    """The 16-bit stream copy built from the YET by indexing."""
    N = yet.n_trials
    C = yet.catalogue_size
    P = (C + 65535) >> 16
    NG = (N + G - 1) // G
    ids = yet.ids.astype(np.int64)
    lengths = np.diff(yet.offsets)
    t_of = np.repeat(np.arange(N, dtype=np.int64), lengths)
    q = ids >> 16
    g = t_of // G
    order = np.lexsort((np.arange(ids.shape[0]), t_of, q))       # part, then trial, then time
    cnt = np.bincount(q * NG + g, minlength=P * NG).reshape(P, NG)
    padded = (cnt + 7) & ~7
    gstart = np.zeros((P, NG + 1), dtype=np.int64)
    np.cumsum(padded, axis=1, out=gstart[:, 1:])
    base = np.zeros(P + 1, dtype=np.int64)
    np.cumsum(gstart[:, NG], out=base[1:])
    key = (q * NG + g)[order]
    first = np.searchsorted(key, key, side="left")
    pos = base[q[order]] + gstart[q[order], g[order]] + (np.arange(key.shape[0]) - first)
    stream = np.full(base[P], 0xFFFF, dtype=np.uint16)
    stream[pos] = (ids[order] & 0xFFFF).astype(np.uint16)
    # trial ends inside each group, per part (slots past the group repeat its end)
    tq = np.bincount(t_of * P + q, minlength=N * P).reshape(N, P)
    tq_pad = np.zeros((NG * G, P), dtype=np.int64)
    tq_pad[:N] = tq
    ends = np.cumsum(tq_pad.reshape(NG, G, P), axis=1)             # [NG][G][P]
    gend = np.zeros((P, NG, 64), dtype=np.int64)
    gend[:, :, :G] = ends.transpose(2, 0, 1)
    gend[:, :, G:] = gend[:, :, G - 1:G]
    return stream, base, gstart, gend


def _check_stream(ara, tables, yet):
    lay = tables.layout()
    G = lay["stream_group_trials"]
    assert 16 <= G <= 63 and lay["stream_parts"] == (yet.catalogue_size + 65535) >> 16
    stream, base, gstart, gend = _expected_stream(yet, G)
    assert lay["stream_ids"] == stream.shape[0]
    assert np.array_equal(ara.debug_read(tables, ara.DEBUG_STREAM_IDS), stream)
    assert np.array_equal(ara.debug_read(tables, ara.DEBUG_STREAM_BASE), base)
    assert np.array_equal(ara.debug_read(tables, ara.DEBUG_STREAM_GSTART).astype(np.int64), gstart.ravel())
    assert np.array_equal(ara.debug_read(tables, ara.DEBUG_STREAM_GEND).astype(np.int64), gend.ravel())


def test_stream_copy_is_the_yet(ara):
    """config0 (two parts), a 20-part catalogue with ragged trials, and trials
    of 0-3 events (groups of 63, mostly empty segments)."""
    w = make_config("config0")
    for yet in (w.yet, make_yet(3000, 150.0, 1_300_000, seed=183), make_yet(5000, 1.5, 300_000, seed=184)):
        pool = make_elt_pool(1, yet.catalogue_size, 10, seed=185)
        tables = ara.create_tables(yet.offsets, yet.ids, pool.losses)
        _check_stream(ara, tables, yet)
        tables.close()


def test_stream_copy_groups_past_the_stage(ara):
    """Groups whose padded segments exceed the scatter's LDS stage are written
    to the stream directly: trials of ~5000 events (every group too large),
    and long trials followed by short ones (both kinds in one layout)."""
    rng = np.random.default_rng(187)
    C = 2_000_000
    lengths = np.concatenate([rng.integers(4000, 7000, 100), rng.integers(0, 50, 3000)])
    trials = [rng.integers(0, C, size=int(k)).tolist() for k in lengths]
    for yet in (make_yet(600, 5000.0, 300_000, seed=186), make_tiny_yet(trials, C)):
        pool = make_elt_pool(1, yet.catalogue_size, 10, seed=188)
        tables = ara.create_tables(yet.offsets, yet.ids, pool.losses)
        _check_stream(ara, tables, yet)
        tables.close()


def test_stream_copy_config1_prefix(ara):
    """The first 20 000 trials of the 1M-trial workload: 31 parts of 2^16
    events, about 32 events per (trial, part)."""
    w = make_config("config1", n_prefix=20_000)
    tables = ara.create_tables(w.yet.offsets, w.yet.ids, w.pool.losses)
    _check_stream(ara, tables, w.yet)
    tables.close()
