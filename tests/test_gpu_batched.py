"""GPU parity of the ragged batched path (CSR and row-table forms, with and
without hipGraph replay) against the FP64 oracle, through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2207_00257_amd import _lib as L
from paper_2207_00257_amd import api, synth
from parity_util import assert_f32_close, assert_within_ulp, bf16_bits_to_f64, ulp_bf16

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def run_csr(x, offs, ctx=None, accum="f32", out_dtype=torch.float32):
    inp = gpu(x)
    out = torch.full((x.size,), -7.0, dtype=out_dtype, device=DEV)
    api.normalize_batched(out, inp, gpu(offs), accum=accum, ctx=ctx)
    torch.cuda.synchronize()
    return out


def check_rows(got, x, offs, what=""):
    ref = oracle.normalize_batched(x, offs)
    covered = np.zeros(x.size, bool)
    for r in range(offs.size - 1):
        covered[offs[r]:offs[r + 1]] = True
    assert_f32_close(got[covered], ref[covered], what=what)
    return covered


def test_golden_three_rows_one_empty():
    x = np.array([1, 3, 1, 1, 2], np.float32)
    offs = np.array([0, 2, 2, 5], np.int64)
    got = run_csr(x, offs).cpu().numpy()
    assert list(got) == [0.25, 0.75, 0.25, 0.25, 0.5]


LENGTHS = [0, 1, 2, 3, 31, 32, 33, 0, 1000, 4095, 4096, 4097, 8191, 8192, 8193, 65535, 65536, 65537,
           300_001, 1, 0, 1 << 20, 7]


@pytest.mark.parametrize("accum", ["f32", "kahan"])
def test_mixed_lengths_short_and_tiled(accum):
    lengths = np.array(LENGTHS, np.int64)
    offs = synth.ragged_offsets(lengths)
    x = synth.lognormal_f32(int(offs[-1]), 50, 1.0)
    ctx = api.Context()
    got = run_csr(x, offs, ctx, accum=accum).cpu().numpy()
    check_rows(got, x, offs, "mixed lengths " + accum)
    assert ctx.device_error() == L.NRM_OK
    ctx.close()


BATCH_PARAMS = [
    dict(),
    dict(graph=0),                      # the kernels launched one by one
    dict(block=64, unroll=1, map_unroll=1, short_regs=1, tile_log2=10, grid=7),
    dict(block=1024, unroll=8, map_unroll=8, short_regs=8, tile_log2=20, grid=256),
    dict(block=512, unroll=2, map_unroll=4, short_regs=2, tile_log2=14, grid=3000),
    dict(block=128, unroll=4, map_unroll=2, short_regs=4, tile_log2=12, grid=1),
    dict(graph=1),
    dict(graph=1, block=512, tile_log2=18, short_regs=4),
    dict(map_block=64, map_grid=3, map_unroll=8),
    dict(map_block=1024, map_grid=5000, tile_log2=11, grid=64),
    dict(keep_mib=0),                   # every tile non-temporal
    dict(keep_mib=1, tile_log2=10),     # the last 256 tiles temporal, the rest not
    dict(keep_mib=4096, graph=1),       # every tile temporal
    dict(resident_segments=0, wave_max=0),  # single-pass rows and tiles only
    dict(resident_segments=0),          # short rows one per wavefront, single-pass rows and tiles
    dict(resident_segments=1, resident_grid=3, wave_max=0),  # one-segment resident rows, the rest tiled
    dict(resident_segments=3, resident_grid=5, graph=1),
    dict(resident_segments=64, resident_grid=64, tile_log2=11),
    dict(wave_max=0),                   # no short rows' kernel: resident rows down to n = 1
    dict(wave_max=1, wave_grid=1),      # one block of four wavefronts, rows of one element only
    dict(wave_max=100, wave_grid=3, graph=1),
    dict(wave_max=2048, wave_grid=5000),  # more wavefronts than rows
]


@pytest.mark.parametrize("params", BATCH_PARAMS, ids=lambda p: ",".join("%s=%s" % kv for kv in p.items()) or "default")
def test_launch_parameters(params):
    ctx = api.Context()
    ctx.set_batch_params(**params)
    lengths = synth.loguniform_lengths(300, 51, 1, 1 << 17)
    lengths[::17] = 0
    offs = synth.ragged_offsets(lengths)
    x = synth.lognormal_f32(int(offs[-1]), 52, 1.0)
    got = run_csr(x, offs, ctx).cpu().numpy()
    check_rows(got, x, offs, str(params))
    assert ctx.device_error() == L.NRM_OK
    ctx.close()


def test_batch_parameter_validation():
    ctx = api.Context()
    good = ctx.get_batch_params()
    for bad in (dict(block=96), dict(map_block=2048), dict(unroll=3), dict(map_unroll=16), dict(short_regs=0),
                dict(grid=0), dict(map_grid=0), dict(tile_log2=9), dict(tile_log2=23), dict(graph=2),
                dict(keep_mib=-1), dict(keep_mib=4097), dict(resident_segments=-1), dict(resident_segments=65),
                dict(resident_segments=4, resident_grid=0), dict(resident_segments=8, resident_grid=4),
                dict(wave_max=-1), dict(wave_max=2049), dict(wave_grid=0), dict(wave_grid=(1 << 20) + 1)):
        with pytest.raises(L.NrmError):
            ctx.set_batch_params(**bad)
        assert ctx.get_batch_params() == good, bad
    p = L.NrmBatchParams()
    assert L.lib().nrm_default_batch_params(ctypes.byref(p)) == L.NRM_OK
    assert {f: getattr(p, f) for f, _ in L.NrmBatchParams._fields_} == good
    p.resident_grid = -1
    assert L.lib().nrm_set_batch_params(ctx.handle, ctypes.byref(p)) == L.NRM_EINVAL
    ctx.close()


def test_graph_replays_with_new_batches_and_eager_work_between():
    """One captured graph replayed for several different batches, with eager
    library calls and synchronizations between the replays; every replay is
    checked against the oracle and against the same batch run eagerly."""
    gctx = api.Context()
    gctx.set_batch_params(graph=1)
    gctx.batch_reserve(512, 1 << 22)
    ectx = api.Context()
    for k in range(4):
        lengths = synth.loguniform_lengths(200 + 50 * k, 60 + k, 1, 1 << 15)
        offs = synth.ragged_offsets(lengths)
        x = synth.lognormal_f32(int(offs[-1]), 70 + k, 1.0)
        g_out = run_csr(x, offs, gctx)
        e_out = run_csr(x, offs, ectx)  # eager work between replays
        check_rows(g_out.cpu().numpy(), x, offs, "graph replay %d" % k)
        assert torch.equal(g_out, e_out), k
        y = synth.uniform_f32(100_000, 80 + k)
        t = gpu(y)
        api.normalize(t, t)  # plain eager call in between
        torch.cuda.synchronize()
    assert gctx.device_error() == L.NRM_OK
    gctx.close()
    ectx.close()


def test_row_is_position_independent():
    """A row's bits depend on its length, alignment and dtypes only: the same
    row alone, or at another place in another batch (same 128-byte alignment),
    gives identical bits."""
    ctx = api.Context()
    row = synth.lognormal_f32(100_000, 90, 1.0)  # a multiple of 32: the next row stays aligned
    short = synth.lognormal_f32(3001, 91, 1.0)
    alone = run_csr(row, np.array([0, row.size], np.int64), ctx).cpu().numpy()
    alone_s = run_csr(short, np.array([0, short.size], np.int64), ctx).cpu().numpy()
    filler = synth.lognormal_f32(32 * 1543, 92, 1.0)  # a multiple of 32 floats: same alignment after it
    x = np.concatenate([filler, row, short, filler])
    offs = np.array([0, 7, filler.size, filler.size + row.size, filler.size + row.size + short.size, x.size],
                    np.int64)
    got = run_csr(x, offs, ctx).cpu().numpy()
    assert np.array_equal(got[filler.size:filler.size + row.size], alone)
    assert np.array_equal(got[filler.size + row.size:filler.size + row.size + short.size], alone_s)
    ctx.close()


def test_bad_offsets_are_flagged_and_skipped():
    """Decreasing, negative or out-of-capacity rows are skipped on the device
    (never read or written) and reported; valid rows are still computed."""
    x = synth.lognormal_f32(1000, 93, 1.0)
    ctx = api.Context()
    offs = np.array([0, 100, -5, 300, 1000], np.int64)  # row 1 decreasing, row 2 negative start
    got = run_csr(x, offs, ctx).cpu().numpy()
    assert ctx.device_error() == L.NRM_EDEVICE
    assert ctx.device_error() == L.NRM_OK  # cleared
    assert_f32_close(got[:100], oracle.normalize(x[:100]), what="row 0")
    assert np.all(got[100:300] == -7.0)
    assert_f32_close(got[300:1000], oracle.normalize(x[300:1000]), what="row 3")
    # a row ending past the buffer is skipped, the buffer outside rows untouched
    inp = gpu(x)
    out = torch.full((1000,), -7.0, device=DEV)
    bad = gpu(np.array([0, 500, 1200], np.int64))
    api.normalize_batched(out, inp, bad, ctx=ctx)
    assert ctx.device_error() == L.NRM_EDEVICE
    o = out.cpu().numpy()
    assert_f32_close(o[:500], oracle.normalize(x[:500]), what="valid row")
    assert np.all(o[500:] == -7.0)
    ctx.close()


@pytest.mark.parametrize("reserve", [0, 20000], ids=["one_launch_planner", "split_planner"])
def test_bad_rows_in_later_planner_rounds(reserve):
    """Each round of 1024 rows is planned by its own block: invalid rows in
    rounds 1 and 3 are flagged and skipped by their owners while every valid
    row of every round is computed. With room for more than 4096 rows the
    planner is split (a counting launch first); the result is the same."""
    lengths = synth.loguniform_lengths(3100, 95, 1, 3000)
    lengths[[7, 2049, 3098]] = [70_000, 50_000, 90_000]  # long rows in rounds 0, 2 and 3
    offs = synth.ragged_offsets(lengths)
    x = synth.lognormal_f32(int(offs[-1]), 96, 1.0)
    bad = offs.copy()
    bad[1500] = -5          # row 1499 ends before it starts, row 1500 starts below zero
    bad[3080] = x.size + 9  # row 3079 ends past the buffer, row 3080 starts past its end
    ctx = api.Context()
    if reserve:
        ctx.batch_reserve(reserve, x.size)
    got = run_csr(x, bad, ctx).cpu().numpy()
    assert ctx.device_error() == L.NRM_EDEVICE
    assert ctx.device_error() == L.NRM_OK  # cleared
    skipped = {1499, 1500, 3079, 3080}
    for r in range(lengths.size):
        b, e = int(offs[r]), int(offs[r + 1])
        if r in skipped:
            assert np.all(got[b:e] == -7.0), r
        elif e > b:
            assert_f32_close(got[b:e], oracle.normalize(x[b:e]), what="row %d" % r)
    ctx.close()


def test_graph_with_spare_planner_blocks():
    """A graph captured for a workspace of 8192 rows (eight planner blocks)
    replayed for batches of 3100, 10 and 1024 rows: the blocks past each
    batch's last round return at once, every row is computed."""
    ctx = api.Context()
    ctx.set_batch_params(graph=1)
    ctx.batch_reserve(8192, 1 << 23)
    for rows, seed in ((3100, 97), (10, 98), (1024, 99), (3100, 100)):
        lengths = synth.loguniform_lengths(rows, seed, 1, 1 << 13)
        lengths[::13] = 0
        offs = synth.ragged_offsets(lengths)
        x = synth.lognormal_f32(int(offs[-1]), seed + 50, 1.0)
        check_rows(run_csr(x, offs, ctx).cpu().numpy(), x, offs, "%d rows" % rows)
        assert ctx.device_error() == L.NRM_OK
    ctx.close()


def test_rows_table_mixed_dtypes():
    """Row-table form: each row has its own buffers and dtypes."""
    specs = [("f32", "f32", 5000), ("bf16", "bf16", 70_000), ("f16", "f32", 1234), ("bf16", "f32", 200_000),
             ("f32", "bf16", 33), ("f32", "f32", 1 << 18), ("f32", "f32", 0), ("f16", "f16", 3000)]
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
    pairs, refs, infos = [], [], []
    for i, (di, do, n) in enumerate(specs):
        v = synth.lognormal_f32(n, 100 + i, 1.0)
        if di == "f32":
            host, odt = v, "f32"
        elif di == "bf16":
            host, odt = synth.f32_to_bf16_bits(v), "bf16"
        else:
            host, odt = synth.f32_to_f16_bits(v), "f16"
        inp = gpu(host.view(np.int16) if di != "f32" else host)
        if di != "f32":
            inp = inp.view(tdt[di])
        out = torch.empty(n, dtype=tdt[do], device=DEV)
        pairs.append((out, inp))
        refs.append(oracle.normalize(host, odt) if n else np.zeros(0))
        infos.append((di, do, n))
    ctx = api.Context()
    ctx.normalize_rows(pairs)
    torch.cuda.synchronize()
    for (out, _), ref, (di, do, n) in zip(pairs, refs, infos):
        if n == 0:
            continue
        if do == "f32":
            assert_f32_close(out.cpu().numpy(), ref, what="%s->%s n=%d" % (di, do, n))
        elif do == "bf16":
            got = bf16_bits_to_f64(out.view(torch.int16).cpu().numpy().view(np.uint16))
            assert_within_ulp(got, ref, ulp_bf16, what="%s->bf16 n=%d" % (di, n))
        else:
            from parity_util import ulp_f16
            assert_within_ulp(out.cpu().numpy().astype(np.float64), ref, ulp_f16, what="%s->f16" % di)
    assert ctx.device_error() == L.NRM_OK
    ctx.close()


def test_rows_table_graph_replay_same_as_alone():
    """Rows in a graph-replayed table batch equal the same rows run alone
    (batch of one), bit for bit."""
    ctx = api.Context()
    ctx.set_batch_params(graph=1)
    ctx.batch_reserve(64, 1 << 22)
    xs = [synth.lognormal_f32(n, 110 + i, 1.0) for i, n in enumerate([10, 5000, 70_000, 300_000, 2048])]
    ins = [gpu(v) for v in xs]
    outs = [torch.empty_like(t) for t in ins]
    ctx.normalize_rows(list(zip(outs, ins)))
    torch.cuda.synchronize()
    for v, t_in, t_out in zip(xs, ins, outs):
        solo = torch.empty_like(t_in)
        ctx.normalize_rows([(solo, t_in)])
        torch.cuda.synchronize()
        assert torch.equal(solo, t_out)
        assert_f32_close(t_out.cpu().numpy(), oracle.normalize(v), what="n=%d" % v.size)
    ctx.close()


def test_misaligned_output_rows():
    """Output buffer offset by one element from the input's alignment: the
    element-wise store path."""
    lengths = np.array([5, 5000, 100_000, 3], np.int64)
    offs = synth.ragged_offsets(lengths)
    x = synth.lognormal_f32(int(offs[-1]), 120, 1.0)
    inp = gpu(x)
    big = torch.full((x.size + 1,), -7.0, device=DEV)
    out = big[1:]
    api.normalize_batched(out, inp, gpu(offs))
    torch.cuda.synchronize()
    got = big.cpu().numpy()
    assert got[0] == -7.0
    check_rows(got[1:], x, offs, "misaligned out")


def test_ragged_4096_rows_full_workload():
    """The ragged benchmark workload: 4096 rows, lengths log-uniform in
    [32, 2^20], LogNormal(0,1) FP32 values; every element against the oracle,
    in the launch configuration the benchmark times (the tuned entry, else the
    defaults), through a captured graph."""
    from paper_2207_00257_amd import tune

    x, offs = synth.ragged_batch(4096, 4)
    ctx = api.Context()
    ctx.set_batch_params(**dict(tune.load_batch_params() or {}, graph=1))
    got = run_csr(x, offs, ctx).cpu().numpy()
    assert ctx.device_error() == L.NRM_OK
    ref = oracle.normalize_batched(x, offs)
    assert_f32_close(got, ref, what="4096 ragged rows")
    ctx.close()


def test_workspace_grows_between_calls():
    ctx = api.Context()
    for rows, hi, seed in ((10, 1000, 130), (2000, 1 << 16, 131), (5, 1 << 21, 132)):
        lengths = synth.loguniform_lengths(rows, seed, 1, hi)
        offs = synth.ragged_offsets(lengths)
        x = synth.lognormal_f32(int(offs[-1]), seed, 1.0)
        check_rows(run_csr(x, offs, ctx).cpu().numpy(), x, offs, "rows=%d" % rows)
    ctx.close()


def test_rows_with_many_tiles():
    """Rows of more than 64 and more than 1024 tiles: the row sum merges its
    partials in one wavefront, then through the LDS tree."""
    ctx = api.Context()
    ctx.set_batch_params(tile_log2=10, block=64, unroll=1, map_unroll=1)
    lengths = np.array([70 * 1024 + 5, 3, 1100 * 1024 + 17, 5000], np.int64)
    offs = synth.ragged_offsets(lengths)
    x = synth.lognormal_f32(int(offs[-1]), 140, 1.0)
    check_rows(run_csr(x, offs, ctx).cpu().numpy(), x, offs, "many tiles")
    assert ctx.device_error() == L.NRM_OK
    ctx.close()


@pytest.mark.parametrize("seed", range(12))
def test_random_batches_match_oracle(seed):
    """Seeded random batches: row counts up to 3000 (one to three planner
    rounds), lengths drawn around the boundaries the scheduler has (empty,
    one element, the single-pass limit, whole tiles and one element either
    side), random launch shapes, graph replay or not."""
    rng = np.random.default_rng(1000 + seed)
    shapes = [dict(), dict(block=64, unroll=1, map_unroll=1, short_regs=1, tile_log2=10, grid=7, resident_segments=0,
                           graph=0),
              dict(block=512, unroll=2, short_regs=2, tile_log2=13, map_grid=33, resident_segments=2),
              dict(graph=1, tile_log2=12, resident_segments=5, resident_grid=9),
              dict(keep_mib=0, map_block=256, map_unroll=8, grid=100, resident_segments=0),
              dict(graph=1, resident_segments=64)]
    params = shapes[seed % len(shapes)]
    ctx = api.Context()
    ctx.set_batch_params(**params)
    bp = ctx.get_batch_params()
    seg = 1 << 14  # elements of one resident segment
    short_max = (bp["resident_segments"] * seg if bp["resident_segments"] else
                 bp["block"] * bp["short_regs"] * 4)
    tile = 1 << bp["tile_log2"]
    edges = np.array([0, 1, 2, short_max - 1, short_max, short_max + 1, tile - 1, tile, tile + 1, 2 * tile + 3,
                      3 * tile, seg - 1, seg, seg + 1, 2 * seg + 1], np.int64)
    rows = int(rng.integers(1, 3001))
    kind = rng.integers(0, 3, rows)
    lengths = np.where(kind == 0, rng.choice(edges, rows), rng.integers(0, 3 * short_max, rows))
    lengths[kind == 2] = rng.integers(short_max, max(6 * tile, 2 * short_max), int((kind == 2).sum()))
    while lengths.sum() > 12_000_000:  # keep the oracle quick
        lengths //= 2
    offs = synth.ragged_offsets(lengths)
    x = synth.lognormal_f32(int(offs[-1]), 2000 + seed, 1.0)
    check_rows(run_csr(x, offs, ctx).cpu().numpy(), x, offs, "seed %d %s rows=%d" % (seed, params, rows))
    assert ctx.device_error() == L.NRM_OK
    ctx.close()


def test_many_rows_planner_rounds():
    """More rows than the planner's threads (several scan rounds), with empty,
    short and long rows interleaved."""
    lengths = synth.loguniform_lengths(5000, 141, 1, 1 << 14)
    lengths[::7] = 0
    lengths[3::11] = 40000
    offs = synth.ragged_offsets(lengths)
    x = synth.lognormal_f32(int(offs[-1]), 142, 1.0)
    ctx = api.Context()
    check_rows(run_csr(x, offs, ctx).cpu().numpy(), x, offs, "5000 rows")
    assert ctx.device_error() == L.NRM_OK
    ctx.close()


RESIDENT_LENGTHS = [1, (1 << 14) - 1, 1 << 14, (1 << 14) + 1, 2 * (1 << 14) + 5, 0, 63 * (1 << 14) + 3,
                    1 << 20, (1 << 20) + 1, 37, 5 * (1 << 14)]


@pytest.mark.parametrize("accum", ["f32", "kahan"])
def test_resident_rows_across_segment_boundaries(accum):
    """Rows held on chip between their read and their write, with lengths at
    the segment boundaries (2^14 elements), up to the 64-segment limit (2^20)
    and one past it (a tiled row), at misaligned starts; then the same rows
    with the resident path off: both within the bound of the oracle."""
    lengths = np.array(RESIDENT_LENGTHS, np.int64)
    offs = synth.ragged_offsets(lengths) + 3  # every row starts 12 bytes past a line
    x = synth.lognormal_f32(int(offs[-1]), 150, 1.0)
    for seg in (64, 0):
        ctx = api.Context()
        ctx.set_batch_params(resident_segments=seg)
        got = run_csr(x, offs, ctx, accum=accum).cpu().numpy()
        check_rows(got, x, offs, "resident_segments=%d %s" % (seg, accum))
        assert ctx.device_error() == L.NRM_OK
        ctx.close()


def test_resident_rows_repeat_bitwise_and_position_independent():
    """A resident row's result depends only on its length and alignment: the
    same row alone, in a batch, and on a later call (the tags of the earlier
    call's partials must not be taken for this call's) gives the same bits."""
    n = 7 * (1 << 14) + 11
    row = synth.lognormal_f32(n, 151, 1.0)
    ctx = api.Context()
    ctx.set_batch_params(graph=1)
    alone = run_csr(row, np.array([0, n], np.int64), ctx).cpu().numpy()
    other = synth.lognormal_f32(3 * (1 << 14) + 64, 152, 1.0)
    x = np.concatenate([other, row, other])
    offs = np.array([0, other.size, other.size + n, x.size], np.int64)
    for _ in range(3):
        got = run_csr(x, offs, ctx).cpu().numpy()
        assert np.array_equal(got[other.size:other.size + n].view(np.uint32), alone.view(np.uint32))
    assert ctx.device_error() == L.NRM_OK
    ctx.close()


def test_back_to_back_calls_do_not_block_the_host():
    """Three batched calls enqueued back to back on one context (CSR form
    with the capacity given, graph replay) return to the host before the
    device has finished the first: the per-call staging buffers are used in
    turn, so no call waits on the one before. GPU time from events; every
    output against the oracle."""
    import time

    x, offs = synth.ragged_batch(4096, 4)
    ref = oracle.normalize_batched(x, offs)
    inp, o = gpu(x), gpu(offs)
    outs = [torch.full_like(inp, -1.0) for _ in range(3)]
    ctx = api.Context()
    ctx.set_batch_params(graph=1)
    for k in range(4):  # every staging buffer's graph captured, workspace sized
        api.normalize_batched(outs[k % 3], inp, o, ctx=ctx)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for t in outs:
        t.fill_(-1.0)
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    for t in outs:
        api.normalize_batched(t, inp, o, ctx=ctx)
    host_ms = (time.perf_counter() - t0) * 1e3
    e1.record(stream)
    torch.cuda.synchronize()
    gpu_ms = e0.elapsed_time(e1)
    print("3 calls: host %.3f ms to enqueue, device %.3f ms" % (host_ms, gpu_ms))
    assert host_ms < gpu_ms / 3, (host_ms, gpu_ms)
    for t in outs:
        assert_f32_close(t.cpu().numpy(), ref, what="back-to-back call")
    assert ctx.device_error() == L.NRM_OK
    ctx.close()


@pytest.mark.parametrize("graph", [0, 1])
def test_split_planner_same_bits_as_one_launch_planner(graph):
    """The same 3000-row batch planned in one launch (room for 4096 rows) and
    by the split planner (room for 50000 rows): identical bits, and the
    oracle's values within the bound."""
    lengths = synth.loguniform_lengths(3000, 160, 1, 1 << 16)
    lengths[::9] = 0
    lengths[5::97] = 300_000  # long rows, tiled
    offs = synth.ragged_offsets(lengths)
    x = synth.lognormal_f32(int(offs[-1]), 161, 1.0)
    outs = []
    for cap in (4096, 50000):
        ctx = api.Context()
        ctx.set_batch_params(graph=graph)
        ctx.batch_reserve(cap, x.size)
        outs.append(run_csr(x, offs, ctx).cpu().numpy())
        assert ctx.device_error() == L.NRM_OK
        ctx.close()
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))
    check_rows(outs[1], x, offs, "split planner")


def test_hundred_thousand_short_rows():
    """A batch of 100000 rows, lengths log-uniform in [1, 3000] (most taken
    one per wavefront, the rest resident), some empty and some long: every
    row against the oracle, through a replayed graph."""
    lengths = synth.loguniform_lengths(100_000, 162, 1, 3000)
    lengths[::31] = 0
    lengths[17::5003] = 200_000
    offs = synth.ragged_offsets(lengths)
    x = synth.lognormal_f32(int(offs[-1]), 163, 1.0)
    ctx = api.Context()
    ctx.set_batch_params(graph=1)
    ctx.batch_reserve(lengths.size, x.size)
    for _ in range(2):  # the second call replays the graph
        got = run_csr(x, offs, ctx).cpu().numpy()
        check_rows(got, x, offs, "100000 rows")
    assert ctx.device_error() == L.NRM_OK
    ctx.close()


WAVE_LENGTHS = [1, 2, 3, 31, 32, 33, 63, 64, 65, 255, 256, 257, 1000, 2047, 2048, 2049, 0, 5]


@pytest.mark.parametrize("shift", [0, 1, 3, 17])
@pytest.mark.parametrize("accum", ["f32", "kahan"])
def test_wave_rows_lengths_and_alignments(shift, accum):
    """Rows around the wavefront path's limits (one vector per lane, the
    2048-element cap and one past it), every start alignment within a line
    through the shift; then the same with wave_max = 100 (rows above it take
    the resident path): all within the bound of the oracle."""
    lengths = np.array(WAVE_LENGTHS, np.int64)
    offs = synth.ragged_offsets(lengths) + shift
    x = synth.lognormal_f32(int(offs[-1]), 164 + shift, 1.0)
    for wave_max in (2048, 100):
        ctx = api.Context()
        ctx.set_batch_params(wave_max=wave_max)
        got = run_csr(x, offs, ctx, accum=accum).cpu().numpy()
        check_rows(got, x, offs, "wave_max=%d shift=%d %s" % (wave_max, shift, accum))
        assert ctx.device_error() == L.NRM_OK
        ctx.close()


def test_wave_rows_every_dtype_pair():
    """Row-table rows of the wavefront path in every input/output dtype pair,
    at lengths from 1 to 2048: FP32 outputs within the stated bound, BF16 and
    FP16 outputs within one ulp of the oracle's rounded value."""
    from parity_util import ulp_f16
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
    pairs, checks = [], []
    seed = 170
    for di in ("f32", "bf16", "f16"):
        for do in ("f32", "bf16", "f16"):
            for n in (1, 7, 64, 333, 2048):
                seed += 1
                v = synth.lognormal_f32(n, seed, 1.0)
                if di == "f32":
                    host = v
                elif di == "bf16":
                    host = synth.f32_to_bf16_bits(v)
                else:
                    host = synth.f32_to_f16_bits(v)
                inp = gpu(host.view(np.int16) if di != "f32" else host)
                if di != "f32":
                    inp = inp.view(tdt[di])
                out = torch.empty(n, dtype=tdt[do], device=DEV)
                pairs.append((out, inp))
                checks.append((out, oracle.normalize(host, di), "%s->%s n=%d" % (di, do, n), do))
    ctx = api.Context()
    ctx.normalize_rows(pairs)
    torch.cuda.synchronize()
    for out, ref, what, do in checks:
        if do == "f32":
            assert_f32_close(out.cpu().numpy(), ref, what=what)
        elif do == "bf16":
            got = bf16_bits_to_f64(out.view(torch.int16).cpu().numpy().view(np.uint16))
            assert_within_ulp(got, ref, ulp_bf16, what=what)
        else:
            assert_within_ulp(out.cpu().numpy().astype(np.float64), ref, ulp_f16, what=what)
    assert ctx.device_error() == L.NRM_OK
    ctx.close()


def test_wave_row_is_position_independent():
    """A row of the wavefront path gives the same bits alone and at another
    place (same 128-byte alignment) in a batch of other rows."""
    ctx = api.Context()
    row = synth.lognormal_f32(1500, 180, 1.0)
    alone = run_csr(row, np.array([0, row.size], np.int64), ctx).cpu().numpy()
    filler = synth.lognormal_f32(32 * 77, 181, 1.0)
    x = np.concatenate([filler, row, filler])
    offs = np.array([0, 5, filler.size, filler.size + row.size, x.size], np.int64)
    got = run_csr(x, offs, ctx).cpu().numpy()
    assert np.array_equal(got[filler.size:filler.size + row.size].view(np.uint32), alone.view(np.uint32))
    ctx.close()
