"""GPU parity of ragged batches: one persistent, graph-replayed launch over
transforms of mixed power-of-two sizes, against the FP64 oracle and against
plain per-size launches of the same data."""
import numpy as np
import pytest

import oracle
import workloads
from fftcheck import SIGN, TOL, from_device, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fftlib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2308_00497_amd as m
    return m


def ragged_oracle(sizes, offsets, re, im, direction):
    """Oracle transform of every item, grouped by size into batched calls."""
    x = re.astype(np.float64) + 1j * im.astype(np.float64)
    out = np.empty_like(x)
    for n in np.unique(sizes):
        idx = np.nonzero(sizes == n)[0]
        rows = np.stack([x[offsets[i]:offsets[i] + n] for i in idx])
        y = oracle.fft(rows, SIGN[direction], threads=8)
        for r, i in enumerate(idx):
            out[offsets[i]:offsets[i] + n] = y[r]
    return out


def per_item_errors(y, ref, sizes, offsets):
    errs = np.empty(len(sizes))
    for i, (n, o) in enumerate(zip(sizes, offsets)):
        errs[i] = oracle.rel_l2(y[o:o + n], ref[o:o + n])
    return errs


def run_ragged(fftlib, sizes, re, im, layout, direction, out=None):
    x = to_device(re, im, layout)
    with fftlib.RaggedPlan(sizes, layout, direction) as plan:
        y = plan.execute(x, out=out)
        desc = plan.describe()
        return from_device(y, layout), desc


def make(sizes, seed):
    sizes = np.asarray(sizes, dtype=np.int64)
    offsets = np.zeros(len(sizes), dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)[:-1]
    re, im = workloads.uniform_complex((int(sizes.sum()),), seed)
    return sizes, offsets, re, im


@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("direction", ["forward", "inverse"])
def test_c4_against_oracle(fftlib, layout, direction):
    """4096 transforms, sizes 2^k with k ~ U{6..16} (seed 4), one launch."""
    sizes, offsets, re, im = workloads.c4()
    y, desc = run_ragged(fftlib, sizes, re, im, layout, direction)
    ref = ragged_oracle(sizes, offsets, re, im, direction)
    errs = per_item_errors(y, ref, sizes, offsets)
    print(f"[parity] C4 ragged {layout} {direction}: max rel-L2 {errs.max():.3e} "
          f"({desc['tiles']} tiles, {desc['workgroups']} workgroups)")
    assert errs.max() <= TOL


def test_c4_matches_per_size_launches(fftlib):
    """The same transforms computed by plain batched plans, one per size, on size-grouped copies."""
    sizes, offsets, re, im = workloads.c4()
    y, _ = run_ragged(fftlib, sizes, re, im, "interleaved", "forward")
    ref = ragged_oracle(sizes, offsets, re, im, "forward")
    for n in np.unique(sizes):
        idx = np.nonzero(sizes == n)[0]
        gr = np.stack([re[offsets[i]:offsets[i] + n] for i in idx])
        gi = np.stack([im[offsets[i]:offsets[i] + n] for i in idx])
        with fftlib.Plan(int(n), len(idx), "interleaved", "forward") as p:
            yp = from_device(p.execute(to_device(gr, gi, "interleaved")), "interleaved").reshape(len(idx), n)
        for r, i in enumerate(idx):
            assert oracle.rel_l2(yp[r], ref[offsets[i]:offsets[i] + n]) <= TOL
            assert oracle.rel_l2(y[offsets[i]:offsets[i] + n], yp[r]) <= 2 * TOL


@pytest.mark.parametrize("layout", ["interleaved", "split"])
def test_every_size_class(fftlib, layout):
    """Every size from 1 to 2^20 (single-pass classes, two- and three-pass transforms), shuffled."""
    rng = np.random.default_rng(41)
    sizes = [1 << k for k in range(0, 21)] + [1 << k for k in rng.integers(0, 14, size=60)]
    sizes = list(rng.permutation(sizes))
    sizes, offsets, re, im = make(sizes, 42)
    for direction in ("forward", "inverse"):
        y, _ = run_ragged(fftlib, sizes, re, im, layout, direction)
        ref = ragged_oracle(sizes, offsets, re, im, direction)
        errs = per_item_errors(y, ref, sizes, offsets)
        worst = int(np.argmax(errs))
        assert errs.max() <= TOL, (layout, direction, int(sizes[worst]), errs.max())


def test_largest_size(fftlib):
    """2^24 among small transforms: three passes with two workspaces."""
    sizes, offsets, re, im = make([64, 1 << 24, 4096, 2], 43)
    y, desc = run_ragged(fftlib, sizes, re, im, "split", "forward")
    ref = ragged_oracle(sizes, offsets, re, im, "forward")
    assert per_item_errors(y, ref, sizes, offsets).max() <= TOL
    assert desc["multi_pass_transforms"] == 1


def test_single_item_and_uniform(fftlib):
    for sizes in ([4096], [256] * 100, [1] * 7, [1 << 16]):
        s, o, re, im = make(sizes, 44)
        y, _ = run_ragged(fftlib, s, re, im, "interleaved", "forward")
        assert per_item_errors(y, ragged_oracle(s, o, re, im, "forward"), s, o).max() <= TOL


def test_graph_replays_and_buffer_changes(fftlib):
    """Replays of the captured graph with eager work and syncs between them, new
    buffers between replays, and in place: every result equals the first."""
    sizes, offsets, re, im = make([1 << k for k in (6, 13, 9, 16, 12, 7, 15)] * 5, 45)
    ref = ragged_oracle(sizes, offsets, re, im, "forward")
    with fftlib.RaggedPlan(sizes, "interleaved", "forward") as plan:
        x = to_device(re, im, "interleaved")
        first = from_device(plan.execute(x), "interleaved")
        assert per_item_errors(first, ref, sizes, offsets).max() <= TOL
        for k in range(4):
            junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
            torch.cuda.synchronize()
            x2 = x.clone() if k % 2 else x
            out = torch.empty_like(x2)
            y = from_device(plan.execute(x2, out=out), "interleaved")
            assert np.array_equal(y, first), k
            del junk
        xi = x.clone()
        y = from_device(plan.execute(xi, out=xi), "interleaved")
        assert np.array_equal(y, first)


def test_ragged_backward_is_adjoint(fftlib):
    sizes, offsets, re, im = make([64, 4096, 1 << 14, 128], 46)
    x = to_device(re, im, "split")
    with fftlib.RaggedPlan(sizes, "split", "forward") as plan:
        y = from_device(plan.backward(x), "split")
    ref = ragged_oracle(sizes, offsets, re, im, "inverse")
    assert per_item_errors(y, ref, sizes, offsets).max() <= TOL


def test_ragged_workspace_override(fftlib):
    sizes, offsets, re, im = make([1 << 14, 64, 1 << 18], 47)
    with fftlib.RaggedPlan(sizes, "interleaved", "forward") as plan:
        nb = plan.workspace_bytes
        assert nb >= ((1 << 14) + (1 << 18)) * 8
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        plan.set_workspace(ws)
        y = from_device(plan.execute(to_device(re, im, "interleaved")), "interleaved")
    assert per_item_errors(y, ragged_oracle(sizes, offsets, re, im, "forward"), sizes, offsets).max() <= TOL


def test_ragged_autotune_and_every_config(fftlib, tmp_path, monkeypatch):
    """FFT_AUTOTUNE=1 times every ragged configuration and caches the winner
    under the batch's size histogram; each configuration, forced through a
    cache file, computes the same transforms to the oracle's tolerance."""
    import json
    sizes, offsets, re, im = make([1 << k for k in (6, 14, 9, 16, 12, 18, 15, 20)] * 3, 48)
    ref = ragged_oracle(sizes, offsets, re, im, "forward")
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("FFT_AUTOTUNE_CACHE", str(cache))
    monkeypatch.setenv("FFT_AUTOTUNE", "1")
    with fftlib.RaggedPlan(sizes, "interleaved", "forward") as plan:
        d = plan.describe()
        y = from_device(plan.execute(to_device(re, im, "interleaved")), "interleaved")
    assert d["source"] == "autotune"
    assert per_item_errors(y, ref, sizes, offsets).max() <= TOL
    entries = json.loads(cache.read_text())["entries"]
    keys = [k for k in entries if "ragged" in k]
    assert len(keys) == 1 and entries[keys[0]] == d["config"]
    monkeypatch.setenv("FFT_AUTOTUNE", "0")
    i = 0
    for p in (8, 7, 6):
        for g in (8, 6, 4):
            for o in (0, 1):
                cfg = f"ragged:p{p}:g{g}:o{o}"
                forced = tmp_path / f"forced{i}.json"
                i += 1
                forced.write_text(json.dumps({"version": 1, "entries": {keys[0]: cfg}}))
                monkeypatch.setenv("FFT_AUTOTUNE_CACHE", str(forced))
                with fftlib.RaggedPlan(sizes, "interleaved", "forward") as plan:
                    d = plan.describe()
                    y = from_device(plan.execute(to_device(re, im, "interleaved")), "interleaved")
                assert d["source"] == "cache" and d["config"] == cfg
                assert per_item_errors(y, ref, sizes, offsets).max() <= TOL, cfg


@pytest.mark.parametrize("cfg", ["ragged:p8:g8:o0:w8", "ragged:p7:g6:o1:w8", "ragged:p6:g4:o0:w16:s13"])
def test_ragged_pipelined_groups(fftlib, cfg):
    """Multi-pass transforms cut into groups of at most w MiB of workspace,
    group g's pass p in level g + p, the workspace a ring of two slots: three-
    and two-pass chains in different groups, single tiles in level 0, both
    layouts and directions; new buffers on the second run reuse the graph.
    (With 16 MiB groups the batch needs its 2^14 transforms among the
    multi-pass ones, the single-pass limit at 2^13, to form two groups.)"""
    sizes, offsets, re, im = make([1 << 20, 1 << 18, 1 << 6, 1 << 18, 1 << 16, 1 << 14, 1 << 18, 1 << 12,
                                   1 << 16, 1 << 16, 1 << 14, 1 << 16, 1 << 9], 49)
    for direction in ("forward", "inverse"):
        ref = ragged_oracle(sizes, offsets, re, im, direction)
        for layout in ("interleaved", "split"):
            with fftlib.RaggedPlan(sizes, layout, direction, config=cfg) as plan:
                d = plan.describe()
                print(f"[case] {cfg} {layout} {direction}: groups {d['groups']} levels {d['levels']}", flush=True)
                assert d["config"] == cfg and d["source"] == "explicit", d
                assert d["groups"] > 1 and d["levels"] >= d["groups"] + 1, d
                # level 0 mixes single-pass tiles with first passes; every later
                # level holds pass tiles only and runs the pass-only kernel
                assert d["pass_only_levels"] == d["levels"] - 1, d
                for rep in range(2):
                    y = from_device(plan.execute(to_device(re, im, layout)), layout)
                    errs = per_item_errors(y, ref, sizes, offsets)
                    print(f"[parity] {cfg} {layout} {direction} rep {rep}: max rel-L2 {errs.max():.3e}", flush=True)
                    assert errs.max() <= TOL, (cfg, layout, direction, rep)


def test_ragged_pipelined_matches_plain_levels(fftlib):
    """The same batch with and without pipelined groups gives the same
    transforms (each to the oracle's tolerance, and to each other)."""
    sizes, offsets, re, im = make([1 << 17, 1 << 15, 1 << 19, 1 << 10, 1 << 15, 1 << 17, 1 << 16], 50)
    ys = {}
    for cfg in ("ragged:p8:g8:o0", "ragged:p8:g8:o0:w8"):
        with fftlib.RaggedPlan(sizes, "split", "forward", config=cfg) as plan:
            ys[cfg] = from_device(plan.execute(to_device(re, im, "split")), "split")
    ref = ragged_oracle(sizes, offsets, re, im, "forward")
    for y in ys.values():
        assert per_item_errors(y, ref, sizes, offsets).max() <= TOL
    a, b = ys.values()
    assert per_item_errors(a, b, sizes, offsets).max() <= TOL


@pytest.mark.parametrize("layout", ["interleaved", "split"])
def test_single_pass_limit(fftlib, layout):
    """2^14 transforms as one single-pass tile each (32 points per thread,
    radix-32 stages, half-width exchanges) by default, or as two passes with
    the limit at 2^13: both to the oracle's tolerance, among single-pass and
    multi-pass neighbours, both directions."""
    rng = np.random.default_rng(53)
    sz = [1 << 14] * 40 + [1 << 13] * 9 + [1 << 15] * 5 + [1 << 6] * 100 + [1 << 12] * 7
    sizes, offsets, re, im = make(list(rng.permutation(sz)), 54)
    for direction in ("forward", "inverse"):
        ref = ragged_oracle(sizes, offsets, re, im, direction)
        ys = []
        for cfg, multi in (("ragged:p8:g8:o1:w128", 5), ("ragged:p8:g8:o1:w128:s13", 45)):
            print(f"[case] single-pass limit {cfg} {layout} {direction}", flush=True)
            with fftlib.RaggedPlan(sizes, layout, direction, config=cfg) as plan:
                d = plan.describe()
                assert d["config"] == cfg and d["multi_pass_transforms"] == multi, d
                y = from_device(plan.execute(to_device(re, im, layout)), layout)
            errs = per_item_errors(y, ref, sizes, offsets)
            print(f"[parity] {cfg} {layout} {direction}: max rel-L2 {errs.max():.3e}", flush=True)
            assert errs.max() <= TOL, (cfg, layout, direction)
            ys.append(y)
        assert per_item_errors(ys[0], ys[1], sizes, offsets).max() <= TOL


def _resident_grid(fftlib, cfg):
    """Persistent workgroups of a full level: a plan with more tiles than can be
    resident reports the grid in its description (no data is transformed)."""
    with fftlib.RaggedPlan(np.full(64 * 4096, 64, dtype=np.int64), "interleaved", "forward", config=cfg) as p:
        return int(p.describe()["workgroups"])


@pytest.mark.parametrize("layout", ["interleaved", "split"])
def test_class_changes_inside_a_workgroup(fftlib, layout):
    """Size mixes dealt so that every persistent workgroup of level 0 runs one
    tile of a class whose transforms span several wavefronts (first-pass tiles
    of 2^15, 2^10 or 2^14 transforms) and then one tile of a class whose transforms
    fit in one wavefront (2^6, or 2^9): the second class's first LDS exchange
    must not overwrite what the first class's last stage is still reading."""
    cfg = "ragged:p8:g8:o1"
    w = _resident_grid(fftlib, cfg)
    mixes = {
        "pass->2^6": [1 << 15] * (w // 4) + [1 << 6] * (64 * w),   # 4 first-pass tiles per 2^15, 64 per 2^6 tile
        "2^10->2^9": [1 << 10] * (4 * w) + [1 << 9] * (8 * w),     # 4 per 2^10 tile, 8 per 2^9 tile
        "2^14->2^6": [1 << 14] * w + [1 << 6] * (64 * w),          # one per 2^14 tile (half-width exchanges)
    }
    for name, sz in mixes.items():
        rng = np.random.default_rng(51)
        sizes, offsets, re, im = make(list(rng.permutation(sz)), 52)
        for direction in ("forward", "inverse"):
            print(f"[case] {name} {layout} {direction} grid {w}", flush=True)
            with fftlib.RaggedPlan(sizes, layout, direction, config=cfg) as plan:
                d = plan.describe()
                assert d["workgroups"] == w, d
                y = from_device(plan.execute(to_device(re, im, layout)), layout)
            ref = ragged_oracle(sizes, offsets, re, im, direction)
            errs = per_item_errors(y, ref, sizes, offsets)
            print(f"[parity] class change {name} {layout} {direction}: max rel-L2 {errs.max():.3e}", flush=True)
            assert errs.max() <= TOL, (name, layout, direction)
