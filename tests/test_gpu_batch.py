"""GPU parity of the batched path (persistent launch inside a cached HIP graph)
and of the autotuner, through the C ABI."""
import os
import sys

import numpy as np
import pytest

import inputs
import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def seg():
    import torch

    assert torch.cuda.is_available(), "GPU tests need the GPU"
    import paper_1912_11494_amd as P

    P.lib()
    return P


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _atlases():
    long_ = synth.make_atlas(synth.AtlasSpec(6, 9, 80.0, 200.0, 6.0, 12.0), 501)
    short = synth.make_atlas(synth.AtlasSpec(11, 10, 20.0, 80.0, 5.0, 8.0), 502)
    return [long_, short]


def _subjects(atl, sizes, seed):
    subs = []
    for i, n in enumerate(sizes):
        spec = synth.SubjectSpec(n, 2.0, (0.2, 0.2))
        subs.append(synth.make_fibers(atl, spec, seed, subject_idx=i) if n else
                    np.zeros((0, 21, 3), np.float32))
    return subs


def _gpu_atlas(seg, at):
    import torch

    d = torch.device("cuda:0")
    return seg.Atlas(torch.from_numpy(at.centroids).to(d), torch.from_numpy(at.bundle_id).to(d),
                     torch.from_numpy(at.thresholds).to(d))


@pytest.mark.parametrize("mode,tile", [("plain", 0), ("bf16", 1), ("fp16", 1), ("bf16_oriented", 0),
                                       ("bf16", 0), ("fp16", 0), ("fp8", 0), ("fp16", 8)])
def test_batch_matches_oracle(seg, mode, tile):
    """Graph-captured flattened launches (plain, oriented, streaming tiles) and
    the per-pair tile-culled route (tile 0 / 8 of bf16, fp16, fp8)."""
    import torch

    atl = _atlases()
    subs = _subjects(atl, [1500, 0, 257, 3001, 64, 777], seed=77)
    d = torch.device("cuda:0")
    ga = [_gpu_atlas(seg, a) for a in atl]
    gf = [torch.from_numpy(f).to(d) for f in subs]
    log(f"batch mode={mode} tile={tile}")
    outs = seg.segment_batch(ga, gf, mode=mode, tile=tile)
    torch.cuda.synchronize()
    for i, f in enumerate(subs):
        for a, at in enumerate(atl):
            lab = outs[i][a][0].cpu().numpy()
            dist = outs[i][a][1].cpu().numpy()
            if len(f) == 0:
                assert lab.size == 0
                continue
            l32, d32, _ = oracle.segment_f32(f, at.centroids, at.bundle_id, at.thresholds)
            assert np.array_equal(lab, l32), (mode, i, a)
            assert np.array_equal(dist, d32), (mode, i, a)
            # the batch equals the one-subject call
            l1, d1 = ga[a].segment(gf[i], mode=mode)
            assert torch.equal(l1.cpu(), outs[i][a][0].cpu())


def test_batch_graph_replay_and_reshape(seg):
    import torch

    atl = _atlases()
    d = torch.device("cuda:0")
    ga = [_gpu_atlas(seg, a) for a in atl]
    subs = _subjects(atl, [900, 1300], seed=5)
    gf = [torch.from_numpy(f).to(d) for f in subs]
    outs = [[(torch.empty(len(f), dtype=torch.int32, device=d),
              torch.empty(len(f), dtype=torch.float32, device=d)) for _ in atl] for f in subs]
    want = [[oracle.segment_f32(f, at.centroids, at.bundle_id, at.thresholds)[0] for at in atl]
            for f in subs]
    for rep in range(4):
        log(f"replay {rep}")
        for o in outs:
            for lab, dist in o:
                lab.fill_(-7)
        seg.segment_batch(ga, gf, mode="bf16", tile=1, outs=outs)
        torch.cuda.synchronize()
        # eager work between replays
        l_e, _ = ga[0].segment(gf[0], mode="plain")
        torch.cuda.synchronize()
        assert np.array_equal(l_e.cpu().numpy(), want[0][0])
        for i in range(2):
            for a in range(2):
                assert np.array_equal(outs[i][a][0].cpu().numpy(), want[i][a]), (rep, i, a)
    # new data in the same buffers: the replay must read it
    new = _subjects(atl, [900, 1300], seed=6)
    for g, f in zip(gf, new):
        g.copy_(torch.from_numpy(f).to(d))
    seg.segment_batch(ga, gf, mode="bf16", tile=1, outs=outs)
    torch.cuda.synchronize()
    for i, f in enumerate(new):
        for a, at in enumerate(atl):
            l32 = oracle.segment_f32(f, at.centroids, at.bundle_id, at.thresholds)[0]
            assert np.array_equal(outs[i][a][0].cpu().numpy(), l32)
    # another shape: recaptured
    subs3 = _subjects(atl, [300, 50, 1200], seed=8)
    gf3 = [torch.from_numpy(f).to(d) for f in subs3]
    outs3 = seg.segment_batch(ga, gf3, mode="plain")
    torch.cuda.synchronize()
    for i, f in enumerate(subs3):
        for a, at in enumerate(atl):
            l32 = oracle.segment_f32(f, at.centroids, at.bundle_id, at.thresholds)[0]
            assert np.array_equal(outs3[i][a][0].cpu().numpy(), l32)


@pytest.mark.parametrize("mode", ["fp16", "fp8"])
def test_batch_culled_graph_replay(seg, mode):
    """The tile-culled batch (all subjects sorted together, one culled pass per
    atlas) replayed from its cached graph: outputs overwritten between replays,
    eager calls in between, then new fibers in the same buffers, then another
    subject layout (a new capture); every result equals the oracle's."""
    import torch

    atl = _atlases()
    d = torch.device("cuda:0")
    ga = [_gpu_atlas(seg, a) for a in atl]
    subs = _subjects(atl, [700, 2100, 333], seed=41)
    gf = [torch.from_numpy(f).to(d) for f in subs]
    outs = [[(torch.empty(len(f), dtype=torch.int32, device=d),
              torch.empty(len(f), dtype=torch.float32, device=d)) for _ in atl] for f in subs]

    def check(cases, outs, ctx):
        for i, f in enumerate(cases):
            for a, at in enumerate(atl):
                l32, d32, _ = oracle.segment_f32(f, at.centroids, at.bundle_id, at.thresholds)
                assert np.array_equal(outs[i][a][0].cpu().numpy(), l32), (ctx, i, a)
                assert np.array_equal(outs[i][a][1].cpu().numpy(), d32), (ctx, i, a)

    for rep in range(3):
        log(f"culled batch {mode} replay {rep}")
        for o in outs:
            for lab, dist in o:
                lab.fill_(-7)
                dist.fill_(-7.0)
        seg.segment_batch(ga, gf, mode=mode, outs=outs)
        torch.cuda.synchronize()
        l_e, _ = ga[1].segment(gf[1], mode=mode)  # eager work between replays
        torch.cuda.synchronize()
        check(subs, outs, f"replay {rep}")
    new = _subjects(atl, [700, 2100, 333], seed=42)
    for g, f in zip(gf, new):
        g.copy_(torch.from_numpy(f).to(d))
    seg.segment_batch(ga, gf, mode=mode, outs=outs)
    torch.cuda.synchronize()
    check(new, outs, "new data")
    subs3 = _subjects(atl, [0, 129, 4000, 1], seed=43)
    gf3 = [torch.from_numpy(f).to(d) for f in subs3]
    outs3 = seg.segment_batch(ga, gf3, mode=mode)
    torch.cuda.synchronize()
    check(subs3, outs3, "new layout")


def test_batch_empty_atlas(seg):
    import torch

    atl = _atlases()
    d = torch.device("cuda:0")
    empty = seg.Atlas(torch.zeros((0, 21, 3), dtype=torch.float32, device=d),
                      torch.zeros(0, dtype=torch.int32, device=d),
                      torch.ones(1, dtype=torch.float32, device=d))
    assert len(empty) == 0
    subs = _subjects(atl, [400], seed=9)
    gf = [torch.from_numpy(subs[0]).to(d)]
    for tile in (1, 0):
        outs = seg.segment_batch([empty, _gpu_atlas(seg, atl[1])], gf, mode="bf16", tile=tile)
        torch.cuda.synchronize()
        assert (outs[0][0][0] == -1).all() and torch.isinf(outs[0][0][1]).all()
        l32 = oracle.segment_f32(subs[0], atl[1].centroids, atl[1].bundle_id,
                                 atl[1].thresholds)[0]
        assert np.array_equal(outs[0][1][0].cpu().numpy(), l32)


def test_autotune_roundtrip(seg, tmp_path):
    import torch

    atl = _atlases()
    d = torch.device("cuda:0")
    ga = _gpu_atlas(seg, atl[1])
    subs = _subjects(atl, [5000], seed=10)
    f = torch.from_numpy(subs[0]).to(d)
    seg.tune_clear()
    for mode in ("plain", "bf16", "dense"):
        tile, ms = seg.autotune(ga, f, mode=mode, reps=2)
        log(f"autotune {mode}: tile {tile} {ms:.3f} ms")
        assert tile > 0 and ms > 0
        lab, dist = ga.segment(f, mode=mode)  # tile 0 now resolves to the tuned tile
        torch.cuda.synchronize()
        l32, d32, _ = oracle.segment_f32(subs[0], atl[1].centroids, atl[1].bundle_id,
                                         atl[1].thresholds)
        assert np.array_equal(lab.cpu().numpy(), l32)
    path = str(tmp_path / "tune.txt")
    seg.tune_save(path)
    lines = open(path).read().split("\n")
    assert len([x for x in lines if x.strip()]) == 3
    seg.tune_clear()
    seg.tune_load(path)
    seg.tune_clear()


@pytest.mark.workloads("batch-16-subjects-x-2-atlases")
def test_batch_full_size_sampled(seg):
    """The batch workload at full size (16 subjects, 37M fibers, two atlases) on
    both routes; the oracle recomputes 150 fibers of every subject."""
    import torch

    wl = "batch-16-subjects-x-2-atlases"
    atl = synth.workload_atlases(wl)
    subs = synth.workload_subjects(wl)
    seed = synth.workload_seed(wl)
    d = torch.device("cuda:0")
    ga = [_gpu_atlas(seg, a) for a in atl]
    rng = np.random.default_rng(39)
    samples, gf = [], []
    for i, sp in enumerate(subs):
        f = inputs.fibers(wl, i)
        idx = np.sort(rng.choice(len(f), 150, replace=False))
        samples.append((idx, f[idx]))
        gf.append(torch.from_numpy(f).to(d))
        del f
    log(f"batch full size: {sum(int(g.shape[0]) for g in gf)} fibers")
    want = [[oracle.segment_f32(sf, at.centroids, at.bundle_id, at.thresholds)[:2] for at in atl]
            for _, sf in samples]
    for mode, tile in (("fp16", 0), ("bf16", 1)):
        log(f"batch full size mode={mode} tile={tile}")
        outs = seg.segment_batch(ga, gf, mode=mode, tile=tile)
        torch.cuda.synchronize()
        for i, (idx, _) in enumerate(samples):
            ti = torch.from_numpy(idx).to(d)
            for a in range(len(atl)):
                lab = outs[i][a][0][ti].cpu().numpy()
                dist = outs[i][a][1][ti].cpu().numpy()
                assert np.array_equal(lab, want[i][a][0]), (mode, i, a)
                assert np.array_equal(dist, want[i][a][1]), (mode, i, a)
        del outs


@pytest.mark.workloads("batch-16-subjects-x-2-atlases")
def test_batch_culled_chunks_match_single_calls(seg):
    """The tile-culled batch splits its subjects into chunks of at most 2^22
    fibers (consecutive subjects; payloads of a chunk stay cached for its
    passes).  Subjects of 2.32M, 1.0M, 0.9M and 2.0M fibers make two chunks of
    two subjects each; every (subject, atlas) output equals the one-subject
    call, itself checked against the oracle elsewhere."""
    import torch

    wl = "batch-16-subjects-x-2-atlases"
    atl = synth.workload_atlases(wl)
    d = torch.device("cuda:0")
    ga = [_gpu_atlas(seg, a) for a in atl]
    f0 = torch.from_numpy(inputs.fibers(wl, 0)).to(d)
    f1 = torch.from_numpy(inputs.fibers(wl, 1)).to(d)
    gf = [f0, f1[:1_000_000], f1[1_000_000:1_900_000], f0[:2_000_000]]
    gf = [g.contiguous() for g in gf]
    log(f"batch chunks: subjects {[int(g.shape[0]) for g in gf]}")
    for mode in ("fp16", "fp8"):
        outs = seg.segment_batch(ga, gf, mode=mode, tile=0)
        torch.cuda.synchronize()
        for i, f in enumerate(gf):
            for a, at in enumerate(atl):
                c = torch.from_numpy(at.centroids).to(d)
                b = torch.from_numpy(at.bundle_id).to(d)
                t = torch.from_numpy(at.thresholds).to(d)
                lab, dist = seg.segment(f, c, b, t, mode=mode)
                torch.cuda.synchronize()
                assert torch.equal(outs[i][a][0], lab), (mode, i, a)
                assert torch.equal(outs[i][a][1], dist), (mode, i, a)
        del outs


@pytest.mark.parametrize("mode", ["fp16", "bf16"])
def test_batch_culled_many_subjects(seg, mode):
    """A tile-culled chunk of more than 16 subjects carries each row's subject
    and index in an extra payload word (a smaller chunk derives them from the
    subjects' first rows): 21 subjects, some empty or tiny, against the
    oracle."""
    import torch

    atl = _atlases()
    sizes = [0 if i % 7 == 3 else 37 * (i % 5) + 1 + 50 * (i % 3) for i in range(21)]
    subs = _subjects(atl, sizes, seed=91)
    d = torch.device("cuda:0")
    ga = [_gpu_atlas(seg, a) for a in atl]
    gf = [torch.from_numpy(f).to(d) for f in subs]
    log(f"batch of {len(subs)} subjects mode={mode}")
    outs = seg.segment_batch(ga, gf, mode=mode, tile=0)
    torch.cuda.synchronize()
    for i, f in enumerate(subs):
        for a, at in enumerate(atl):
            lab = outs[i][a][0].cpu().numpy()
            dist = outs[i][a][1].cpu().numpy()
            if len(f) == 0:
                assert lab.size == 0
                continue
            l32, d32, _ = oracle.segment_f32(f, at.centroids, at.bundle_id, at.thresholds)
            assert np.array_equal(lab, l32), (mode, i, a)
            assert np.array_equal(dist, d32), (mode, i, a)
