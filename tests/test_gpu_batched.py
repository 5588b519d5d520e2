"""Batched products in one persistent, graph-recorded launch, against the CPU oracle."""
import sys

import numpy as np
import pytest

from oracle import reference as ref
from paper_0803_1975_amd import qmm
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("these tests need a GPU")
    return _t


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def make_problems(torch, shapes, seed):
    rng = np.random.default_rng(seed)
    host, dev = [], []
    for p, m, n, k in shapes:
        A = rng.integers(0, p, (m, k), dtype=np.uint8)
        B = rng.integers(0, p, (k, n), dtype=np.uint8)
        dA = torch.from_numpy(A).cuda()
        dB = torch.from_numpy(B).cuda()
        dC = torch.full((m, n), 255, dtype=torch.uint8, device="cuda")
        host.append((A, B, p))
        dev.append((dA, dB, dC, p))
    return host, dev


def check_all(host, dev):
    for i, ((A, B, p), (_, _, dC, _)) in enumerate(zip(host, dev)):
        np.testing.assert_array_equal(dC.cpu().numpy(), ref.modmul(A, B, p), err_msg=f"product {i}")


EDGE_SHAPES = [(7, 1, 1, 1), (3, 16, 16, 16), (101, 17, 33, 5), (2, 513, 31, 70), (251, 64, 64, 64),
               (256, 65, 129, 200), (5, 3, 300, 1), (13, 200, 1, 90), (31, 128, 32, 512), (11, 32, 128, 17),
               (3, 0, 5, 5), (3, 5, 0, 5), (7, 9, 9, 0),
               # operands just over 16 bytes, and last segments that end past the data
               # (raw tiles pull such loads back inside it and shift the bytes down)
               (11, 16, 16, 1), (7, 20, 20, 3), (101, 33, 17, 15), (3, 130, 67, 129), (5, 2, 9, 9)]


@pytest.mark.parametrize("flags", [0, qmm.BATCH_SHAPE_64x64, qmm.BATCH_SHAPE_32x128, qmm.BATCH_SHAPE_128x32,
                                   qmm.BATCH_SHAPE_128x128, qmm.BATCH_FORCE_FP64, qmm.BATCH_INT8_ONLY,
                                   qmm.BATCH_INT8_ONLY | qmm.BATCH_SHAPE_128x128, qmm.BATCH_RAW,
                                   qmm.BATCH_RAW | qmm.BATCH_SHAPE_64x64, qmm.BATCH_RAW | qmm.BATCH_SHAPE_32x128,
                                   qmm.BATCH_RAW | qmm.BATCH_SHAPE_128x32, qmm.BATCH_RAW | qmm.BATCH_SHAPE_128x128])
def test_batched_edge_shapes(torch, flags):
    note("edge", flags)
    host, dev = make_problems(torch, EDGE_SHAPES, 10 + flags)
    batch = qmm.batched_create(dev, flags)
    try:
        batch.run()
        torch.cuda.synchronize()
        check_all(host, dev)
        for i, (p, m, n, k) in enumerate(EDGE_SHAPES):
            pl = batch.plan(i)
            assert pl.p == p
            if flags & qmm.BATCH_FORCE_FP64:
                want = qmm.PATH_FP64_QADIC
            elif p <= 8 and not flags & (qmm.BATCH_INT8_ONLY | qmm.BATCH_RAW):
                want = qmm.PATH_FP4                   # every edge k here is one exact FP32 block
            else:
                want = qmm.PATH_INT8
            assert pl.path == want, (i, p, flags)
    finally:
        batch.destroy()


@pytest.mark.parametrize("flags", [0, qmm.BATCH_RAW])
def test_graph_replays_match_eager_results(torch, flags):
    shapes = synth.batched_shapes(count=300, seed=7)
    host, dev = make_problems(torch, shapes, 7)
    batch = qmm.batched_create(dev, flags)
    try:
        for replay in range(4):
            note("replay", flags, replay)
            for _, _, dC, _ in dev:
                dC.zero_()                              # eager work between replays
            torch.cuda.synchronize()
            batch.run()
            torch.cuda.synchronize()
            check_all(host, dev)
    finally:
        batch.destroy()


def test_batched_workload_2000_products(torch):
    shapes = synth.batched_shapes()
    assert len(shapes) == 2000
    inputs = synth.batched_inputs(shapes)
    dev = []
    for (p, m, n, k), (A, B) in zip(shapes, inputs):
        dev.append((torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(),
                    torch.full((m, n), 255, dtype=torch.uint8, device="cuda"), p))
    for flags in (0, qmm.BATCH_INT8_ONLY, qmm.BATCH_FORCE_FP64, qmm.BATCH_RAW):
        note("workload", flags)
        batch = qmm.batched_create(dev, flags)
        try:
            batch.run()
            torch.cuda.synchronize()
            for i, ((p, m, n, k), (A, B)) in enumerate(zip(shapes, inputs)):
                np.testing.assert_array_equal(dev[i][2].cpu().numpy(), ref.modmul(A, B, p), err_msg=f"product {i}")
                dev[i][2].fill_(255)
        finally:
            batch.destroy()


def test_autotuner_calibration_and_choices(torch):
    costs = qmm.batched_tune()
    note("costs", costs)
    assert len(costs) == qmm.N_BATCH_COSTS and all(c >= 0 for c in costs) and all(costs[i] > 0 for i in (1, 3, 5, 7))
    qmm.batched_set_costs(costs)
    shapes = [(7, 32, 512, 256), (7, 512, 32, 256), (7, 256, 256, 256), (7, 512, 512, 128)]
    host, dev = make_problems(torch, shapes, 3)
    batch = qmm.batched_create(dev)
    try:
        tiles = [batch.plan(i).tile for i in range(len(shapes))]
        note("tiles", tiles)
        batch.run()
        torch.cuda.synchronize()
        check_all(host, dev)
    finally:
        batch.destroy()


def test_tune_cache_file_gives_the_freshly_tuned_choices(torch, tmp_path, monkeypatch):
    # Calibrate both encodings into a cache file (QMM_TUNE_CACHE), build a batch
    # with the fresh fits; then forget them (empty cache, skewed defaults that would
    # pick other tiles), load the file, and build the batch again: the same tiles,
    # and both batches exact.
    path = str(tmp_path / "tune.json")
    monkeypatch.setenv("QMM_TUNE_CACHE", path)
    qmm.tune_cache_clear()
    ws = torch.empty(qmm.batched_tune_workspace_size(256, 256), dtype=torch.uint8, device="cuda")
    fits = {p: qmm.batched_tune(p, 256, 256, ws=ws) for p in (7, 101)}
    note("fits", fits)
    import json
    doc = json.load(open(path))
    assert {(e["enc"], e["bucket"]) for e in doc["entries"]} >= {("fp4", "le512"), ("int8", "le512")}
    arch = doc["entries"][0]["arch"]
    assert arch.startswith("gfx")
    assert qmm.tune_cache_get(arch, 7, 256, 256) == fits[7] and qmm.tune_cache_get(arch, 101, 300, 300) == fits[101]
    shapes = [(7, 32, 512, 256), (7, 512, 32, 256), (101, 256, 256, 256), (101, 500, 40, 1000), (3, 400, 400, 128),
              (13, 64, 480, 64)]
    host, dev = make_problems(torch, shapes, 21)

    def build_and_run():
        for _, _, dC, _ in dev:
            dC.fill_(255)
        batch = qmm.batched_create(dev)
        try:
            tiles = [batch.plan(i).tile for i in range(len(shapes))]
            batch.run()
            torch.cuda.synchronize()
            check_all(host, dev)
            return tiles
        finally:
            batch.destroy()

    fresh = build_and_run()
    qmm.tune_cache_clear()
    skew = [0.0, 1.0, 50.0, 9.0, 50.0, 9.0, 50.0, 9.0]   # every product on 64 x 64 tiles
    qmm.batched_set_costs(skew)
    try:
        assert build_and_run() == [0] * len(shapes)
        qmm.tune_cache_load(path)
        cached = build_and_run()
    finally:
        qmm.batched_set_costs(fits[101])
        qmm.tune_cache_clear()
    note("tiles", fresh, cached)
    assert cached == fresh


def test_measuring_autotuner_keeps_a_correct_fastest_candidate(torch):
    shapes = synth.batched_shapes(count=200, seed=11)
    host, dev = make_problems(torch, shapes, 11)
    batch = qmm.batched_create(dev, qmm.BATCH_MEASURE)
    try:
        check_all(host, dev)                    # candidates ran on the real buffers
        tiles = {batch.plan(i).tile for i in range(len(shapes))}
        note("measured tiles", tiles)
        assert tiles <= {0, 1, 2, 3}
        for _, _, dC, _ in dev:
            dC.fill_(255)
        batch.run()
        torch.cuda.synchronize()
        check_all(host, dev)
    finally:
        batch.destroy()


def test_batched_rejects_bad_problems(torch):
    A = torch.zeros((4, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(qmm.QmmError):
        qmm.batched_create([(A, A, A, 300)])
    big = torch.zeros((2, 140000), dtype=torch.uint8, device="cuda")
    bigB = torch.zeros((140000, 2), dtype=torch.uint8, device="cuda")
    C = torch.zeros((2, 2), dtype=torch.uint8, device="cuda")
    with pytest.raises(qmm.QmmError) as ei:
        qmm.batched_create([(big, bigB, C, 251)])
    assert ei.value.status == qmm.EUNSUPPORTED


def test_raw_batches_read_strided_operands(torch):
    # raw tiles read A and B in place: operands that are views with padded rows and
    # odd starting columns, C a view too; bytes outside the views stay untouched
    rng = np.random.default_rng(21)
    host, dev, bigs = [], [], []
    for p, m, n, k in [(7, 70, 45, 33), (101, 129, 130, 257), (3, 5, 300, 17), (251, 64, 1, 64)]:
        Ab = rng.integers(0, p, (m, k + 13), dtype=np.uint8)
        Bb = rng.integers(0, p, (k, n + 7), dtype=np.uint8)
        A, B = Ab[:, 5:5 + k], Bb[:, 3:3 + n]
        Cb = torch.full((m + 2, n + 9), 0xEE, dtype=torch.uint8, device="cuda")
        dA = torch.from_numpy(Ab).cuda()[:, 5:5 + k]
        dB = torch.from_numpy(Bb).cuda()[:, 3:3 + n]
        host.append((np.ascontiguousarray(A), np.ascontiguousarray(B), p))
        dev.append((dA, dB, Cb[1:m + 1, 2:n + 2], p))
        bigs.append(Cb)
    batch = qmm.batched_create(dev, qmm.BATCH_RAW)
    try:
        batch.run()
        torch.cuda.synchronize()
        check_all(host, dev)
        for (A, B, p), Cb in zip(host, bigs):
            out = Cb.cpu().numpy()
            m, n = A.shape[0], B.shape[1]
            mask = np.ones_like(out, dtype=bool)
            mask[1:m + 1, 2:n + 2] = False
            assert (out[mask] == 0xEE).all()
    finally:
        batch.destroy()


def test_raw_tiles_at_the_uncentred_bound(torch):
    # Raw tiles use residues below 128 as int8 values without centring while
    # k (p-1)^2 fits int32; all-(p-1) operands at the largest such k, one past it
    # (centred instead), and the moduli on either side of 128.
    cases = [(127, 3, 5, 135266), (127, 3, 5, 135267), (128, 4, 3, 1000), (129, 4, 3, 1000), (2, 1, 1, 70000)]
    host, dev = [], []
    for p, m, n, k in cases:
        A = np.full((m, k), p - 1, dtype=np.uint8)
        B = np.full((k, n), p - 1, dtype=np.uint8)
        host.append((A, B, p))
        dev.append((torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(),
                    torch.empty((m, n), dtype=torch.uint8, device="cuda"), p))
    note("raw uncentred bound", cases)
    batch = qmm.batched_create(dev, qmm.BATCH_RAW)
    try:
        batch.run()
        torch.cuda.synchronize()
        check_all(host, dev)
        for (A, B, p), (_, _, dC, _) in zip(host, dev):
            k = A.shape[1]
            assert (dC.cpu().numpy() == (k * (p - 1) * (p - 1)) % p).all()
    finally:
        batch.destroy()
