"""Batched persistent merge (one captured graph) and the tile-shape autotuner."""
import numpy as np
import pytest
import torch

import oracle.merge as om
from paper_1905_03277_amd import synth, torch_ops
from parity_util import assert_parity

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (frames, H, W, scale, tile, cfa): uneven like the batched workload, small enough for tests
SHAPES = [(8, 96, 128, 1.0, 16, 0), (2, 64, 64, 2.0, 16, 1), (15, 48, 96, 1.5, 8, 0),
          (1, 64, 96, 1.5, 16, 2), (5, 160, 200, 1.0, 32, 3), (3, 70, 102, 2.0, 16, 0),
          (12, 64, 80, 1.0, 16, 0), (4, 128, 96, 1.5, 16, 1)]


def make_bursts():
    out = []
    for i, (n, h, w, s, t, cfa) in enumerate(SHAPES):
        b = synth.make_burst(n, h, w, seed=5000 + i, scale=s, tile_size=t, cfa=cfa)
        out.append(b)
    return out


def as_args(bursts, tunings=None):
    return [(b.frames.to(DEV), b.motion.to(DEV), b.desc, (tunings or {}).get(i, b.tuning))
            for i, b in enumerate(bursts)]


def per_burst(args):
    outs = [torch_ops.merge(f, m, d, t) for f, m, d, t in args]
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def test_batch_equals_per_burst_bitwise_and_replays():
    bursts = make_bursts()
    args = as_args(bursts)
    print("[case] batch of", len(args), flush=True)
    want = per_burst(args)
    outs = torch_ops.merge_batch(args)
    torch.cuda.synchronize()
    for i, (o, w) in enumerate(zip(outs, want)):
        np.testing.assert_array_equal(o.cpu().numpy(), w, err_msg=f"burst {i}")
    # second call replays the captured graph into the same buffers
    for o in outs:
        o.fill_(-1.0)
    torch_ops.merge_batch(args, outs)
    torch.cuda.synchronize()
    for i, (o, w) in enumerate(zip(outs, want)):
        np.testing.assert_array_equal(o.cpu().numpy(), w, err_msg=f"replay burst {i}")
    # new tuning values are uploaded before the replay
    tun = {2: bursts[2].tuning.replace(t=0.5, k_detail=0.4), 4: bursts[4].tuning.replace(s=1.0)}
    args2 = as_args(bursts, tun)
    args2 = [(a[0], a[1], a[2], a2[3]) for a, a2 in zip(args, args2)]   # same buffers
    torch_ops.merge_batch(args2, outs)
    torch.cuda.synchronize()
    want2 = per_burst(args2)
    for i, (o, w) in enumerate(zip(outs, want2)):
        np.testing.assert_array_equal(o.cpu().numpy(), w, err_msg=f"retuned burst {i}")
    assert not np.array_equal(want2[2], want[2])


def test_batch_divergent_fields_bitwise_and_oracle():
    """Displacement fields whose tiles are up to 40 px apart: the merge then
    packs per-alignment-tile windows and the robustness reads its corners
    directly; the persistent batch must still equal the per-burst launches
    bit for bit, and the oracle within the forward tolerance."""
    bursts = make_bursts()[:4]
    rng = np.random.default_rng(71)
    for b in bursts:
        m = b.motion.numpy().copy()
        m[1:] += rng.uniform(-40.0, 40.0, size=m[1:].shape).astype(np.float32)
        m[b.desc.ref_frame] = 0
        b.motion = torch.from_numpy(m)
    args = as_args(bursts)
    print("[case] batch of divergent fields", len(args), flush=True)
    want = per_burst(args)
    outs = torch_ops.merge_batch(args)
    torch.cuda.synchronize()
    for i, (o, w) in enumerate(zip(outs, want)):
        np.testing.assert_array_equal(o.cpu().numpy(), w, err_msg=f"burst {i}")
    b = bursts[0]
    f, m = b.numpy()
    assert_parity(outs[0].cpu().numpy(), om.merge(f, m, b.desc, b.tuning), "divergent batch burst 0")


def test_batch_matches_oracle():
    bursts = make_bursts()
    args = as_args(bursts)
    outs = torch_ops.merge_batch(args)
    torch.cuda.synchronize()
    for i in (1, 2, 5):
        b = bursts[i]
        f, m = b.numpy()
        print("[case] batch member", i, flush=True)
        assert_parity(outs[i].cpu().numpy(), om.merge(f, m, b.desc, b.tuning), f"batch burst {i}")


def test_autotune_picks_a_shape_and_is_used(monkeypatch, tmp_path):
    monkeypatch.setenv("HMFSR_TUNE_CACHE", str(tmp_path / "tune.txt"))
    b = synth.make_burst(6, 192, 256, seed=77, scale=1.5, tile_size=16)
    f, m = b.frames.to(DEV), b.motion.to(DEV)
    v, out = torch_ops.autotune(f, m, b.desc, b.tuning)
    torch.cuda.synchronize()
    assert 0 <= v < 4
    monkeypatch.setenv("HMFSR_MERGE_VARIANT", str(v))
    ref = torch_ops.merge(f, m, b.desc, b.tuning)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())
    monkeypatch.delenv("HMFSR_MERGE_VARIANT")
    again = torch_ops.merge(f, m, b.desc, b.tuning)   # the tuned table now picks v
    torch.cuda.synchronize()
    np.testing.assert_array_equal(again.cpu().numpy(), ref.cpu().numpy())
    lines = (tmp_path / "tune.txt").read_text().split()
    assert lines[-1] == str(v)


def items_per_group(plan):
    """(items, workgroups) of every persistent launch of a batch plan."""
    out = [(plan["robust_items"], plan["robust_groups"])] if plan["robust_items"] else []
    out += [(i, g) for i, g in zip(plan["merge_items"], plan["merge_groups"]) if i]
    return out


@pytest.mark.parametrize("cap", [1, 3, 7])
def test_persistent_loop_few_workgroups_bitwise(cap, monkeypatch):
    """The persistent kernels with their workgroups capped at 1, 3 and 7, so
    that each workgroup pulls many (burst, tile) items in turn, across bursts
    of different frame counts, scales, tile sizes and CFAs, coherent and
    divergent fields: every burst equals its per-burst hmfsr_merge bit for
    bit (every output pixel of Sec. 5.1 is computed independently, so the
    order and grouping of the items cannot matter)."""
    monkeypatch.setenv("HMFSR_BATCH_GROUPS", str(cap))
    bursts = make_bursts()
    rng = np.random.default_rng(300 + cap)
    for b in bursts[::3]:
        m = b.motion.numpy().copy()
        m[1:] += rng.uniform(-40.0, 40.0, size=m[1:].shape).astype(np.float32)
        m[b.desc.ref_frame] = 0
        b.motion = torch.from_numpy(m)
    args = as_args(bursts)
    want = per_burst(args)
    outs = torch_ops.merge_batch(args)
    torch.cuda.synchronize()
    plan = torch_ops.batch_plan(DEV)
    launches = items_per_group(plan)
    print(f"[case] persistent cap {cap}: (items, workgroups) per launch {launches}", flush=True)
    assert launches and all(g == min(cap, i) for i, g in launches)
    # the robustness launch and the largest merge launch: many items per workgroup
    assert launches[0][0] / launches[0][1] >= 3
    assert max(i / g for i, g in launches[1:]) >= 3
    for i, (o, w) in enumerate(zip(outs, want)):
        np.testing.assert_array_equal(o.cpu().numpy(), w, err_msg=f"burst {i}")
    # a replay of the same graph: the counters are reset by the graph itself
    for o in outs:
        o.fill_(-1.0)
    torch_ops.merge_batch(args, outs)
    torch.cuda.synchronize()
    for i, (o, w) in enumerate(zip(outs, want)):
        np.testing.assert_array_equal(o.cpu().numpy(), w, err_msg=f"replay burst {i}")


def test_persistent_loop_full_size_members():
    """A batch mixing a 12 MP x 8 burst at scale 1 and a 3 MP x 15 burst at
    scale 2 (the headline and low-light shapes) with small bursts, at the
    default workgroup count: every persistent launch gives each workgroup at
    least three items. Bitwise equal to per-burst launches; the two large
    members agree with the oracle on sampled windows."""
    from parity_util import assert_parity, oracle_crop
    big = [synth.make_config(2, device=DEV), synth.make_config(3, device=DEV)]
    small = make_bursts()[:3]
    args = [(b.frames, b.motion, b.desc, b.tuning) for b in big] + as_args(small)
    print("[case] full-size batch: per-burst launches", flush=True)
    want = [torch_ops.merge(f, m, d, t) for f, m, d, t in args]
    torch.cuda.synchronize()
    print("[case] full-size batch: graph", flush=True)
    outs = torch_ops.merge_batch(args)
    torch.cuda.synchronize()
    launches = items_per_group(torch_ops.batch_plan(DEV))
    print(f"[case] full-size batch: (items, workgroups) per launch {launches}", flush=True)
    assert launches and all(i / g >= 3 for i, g in launches)
    for i, (o, w) in enumerate(zip(outs, want)):
        assert torch.equal(o, w), f"burst {i} differs from its per-burst launch"
    S = 48
    for b, o in zip(big, outs[:2]):
        f, m = b.numpy()
        OH, OW = o.shape[1:]
        for oy, ox in ((0, OW - S), (OH // 2, OW // 3), (OH - S, OW // 2)):
            print("[case] full-size batch window", b.desc.n_frames, oy, ox, flush=True)
            want_w = oracle_crop(f, m, b.desc, b.tuning, oy, ox, S, S)
            assert_parity(o[:, oy:oy + S, ox:ox + S].cpu().numpy(), want_w, f"batch member window ({oy},{ox})")
