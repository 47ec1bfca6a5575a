"""Uneven batches, kernel variants, the autotuner, FP16 storage in the single-pass kernel,
and graph capture -- on the GPU, against the FP64 oracle and against single-plan calls.

Tolerances as in test_gpu_parity, on relative L2 and on the element-wise error: 1e-5 for
FP32 storage, 1e-3 for FP16 storage (the output's own rounding, 2^-11, dominates).  A batch runs each instance
through the same kernels as a single-plan call, only at other addresses, so the two must
agree bit for bit.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from synth import images as SI
from synth import signals as S
from synth import uneven as U
from parity import worst

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_10291_amd  # noqa: F401
    return torch


def rel(a, b):
    """Relative L2 and element-wise (max-abs over max |b|) error of one result: the larger."""
    return worst(a, b)


def deriv_channels(M):
    return [("deriv", m) for m in range(M)]


def scaled_deriv_tables(M, N):
    """b_m(n) = (i n / N)^m on the default band: derivative channels in units that keep the
    samples of every channel near the signal's own size (FP16 range)."""
    mu = M * N
    n = np.arange(-((mu - 1) // 2), -((mu - 1) // 2) + mu)
    return [(1j * n / N) ** m for m in range(M)]


def oracle_1d(g, M, N, n_out, scaled=False):
    if scaled:
        ch = O.Channels(N=N, kinds=[O.MULT_TABLE] * M, orders=[0] * M, tables=np.stack(scaled_deriv_tables(M, N)))
    else:
        ch = O.Channels(N=N, kinds=[O.MULT_DERIV] * M, orders=list(range(M)))
    return O.reconstruct_1d(ch, g.astype(np.float64), n_out)


# ------------------------------------------------------------------ FP16 single-pass kernel
@pytest.mark.parametrize("N,n_out,M", [(1366, 16384, 3), (2048, 16384, 2), (1022, 8192, 4)])
def test_fused_f16_storage_parity(torch_cuda, N, n_out, M):
    from paper_1802_10291_amd import Plan1D
    g = S.smooth_noisy_batch(0, 3, M, N, 2 * N, dtype=np.float16, deriv_scale=N)
    assert np.isfinite(g).all()
    plan = Plan1D(N=N, n_out=n_out, channels=[("table", t) for t in scaled_deriv_tables(M, N)], storage="f16")
    assert plan.info.path == 1 and plan.variant == "fused_t1"
    y = plan.reconstruct(torch_cuda.from_numpy(g).cuda()).cpu().numpy().astype(np.float64)
    want = oracle_1d(g, M, N, n_out, scaled=True)
    for b in range(3):
        assert rel(y[b], want[b]) <= 1e-3


def test_strided_batch_f16_storage(torch_cuda):
    """The strided call (mci_reconstruct_1d_strided) with FP16 samples and outputs on the
    single-pass kernel: bit-identical to the dense call, the gaps between rows untouched."""
    from paper_1802_10291_amd import Plan1D
    torch = torch_cuda
    N, n_out, M, B = 1366, 16384, 3, 4
    g = torch.from_numpy(S.smooth_noisy_batch(0, B, M, N, 2 * N, dtype=np.float16, deriv_scale=N)).cuda()
    plan = Plan1D(N=N, n_out=n_out, channels=[("table", t) for t in scaled_deriv_tables(M, N)], storage="f16")
    big = torch.zeros((B, M * N + 6), dtype=torch.float16, device="cuda")
    big[:, : M * N] = g.reshape(B, -1)
    out = torch.zeros((B, n_out + 8), dtype=torch.float16, device="cuda")
    yv = out[:, :n_out].unflatten(1, (1, n_out))
    plan.reconstruct(big[:, : M * N].unflatten(1, (M, N)), out=yv)
    assert torch.equal(yv, plan.reconstruct(g))
    assert (out[:, n_out:] == 0).all()


# ------------------------------------------------------------------ variants
def test_every_1d_variant_matches_oracle(torch_cuda):
    from paper_1802_10291_amd import Plan1D
    M, N, n_out = 3, 1366, 16384
    g = S.smooth_noisy_batch(40, 3, M, N, 8192)
    want = oracle_1d(g, M, N, n_out)
    plan = Plan1D(N=N, n_out=n_out, channels=deriv_channels(M))
    names = plan.variants()
    assert names[:3] == ["multipass_r8", "multipass_r4", "fused_t1"]
    gd = torch_cuda.from_numpy(g).cuda()
    for v in names:
        plan.set_variant(v)
        assert plan.variant == v and plan.info.path == (1 if v.startswith("fused") else 0)
        y = plan.reconstruct(gd).cpu().numpy().astype(np.float64)
        for b in range(3):
            assert rel(y[b], want[b]) <= 1e-5, (v, b)
    with pytest.raises(Exception):
        plan.set_variant("line_pass")


@pytest.mark.parametrize("N", [86, 96])      # Bluestein (86 = 2 * 43) and 7-smooth
def test_multipass_radix_variants(torch_cuda, N):
    from paper_1802_10291_amd import Plan1D
    g = S.smooth_noisy_batch(50, 2, 3, N, 4 * N)
    want = oracle_1d(g, 3, N, 4 * 3 * N)
    plan = Plan1D(N=N, n_out=12 * N, channels=deriv_channels(3))
    assert plan.variants() == ["multipass_r8", "multipass_r4", "two_pass"]
    for v in plan.variants():
        plan.set_variant(v)
        y = plan.reconstruct(torch_cuda.from_numpy(g).cuda()).cpu().numpy()
        assert max(rel(y[b], want[b]) for b in range(2)) <= 1e-5, v


@pytest.mark.parametrize("N,n_out,M", [(1024, 4096, 2), (1536, 6144, 2), (96, 1152, 3), (86, 1032, 3),
                                       (4096, 65536, 4), (683, 8192, 3)])
def test_two_pass_transforms_match_oracle(torch_cuda, N, n_out, M):
    """Multi-pass path with its transforms in one or two LDS passes (four-step): lengths that
    factor into line lengths directly (1024 = 32 x 32, 6144 = 96 x 64, 65536 = 256 x 256),
    single-pass lines (96), Bluestein lengths chosen to factor (86 -> 192, 683 -> 1536), and
    a side left on radix passes (1152)."""
    from paper_1802_10291_amd import Plan1D
    g = S.smooth_noisy_batch(60, 3, M, N, 2 * M * N)
    want = oracle_1d(g, M, N, n_out)
    plan = Plan1D(N=N, n_out=n_out, channels=deriv_channels(M))
    plan.set_variant("two_pass")
    y = plan.reconstruct(torch_cuda.from_numpy(g).cuda()).cpu().numpy()
    for b in range(3):
        assert rel(y[b], want[b]) <= 1e-5, b


@pytest.mark.parametrize("N,n_out,M,n1", [(1024, 4096, 2, None), (1536, 6144, 2, None), (86, 1024, 3, None),
                                          (4096, 65536, 4, None), (1366, 16384, 3, 100), (2048, 8192, 3, -5000),
                                          (512, 2048, 2, None), (21846, 262144, 3, None),
                                          (683, 8192, 3, None), (171, 2048, 3, None), (10923, 131072, 3, None)])
def test_real_two_pass_matches_oracle(torch_cuda, N, n_out, M, n1):
    """Real-mode multi-kernel path: rows read as N/2 complex pairs (one pass for 256 and 512,
    two for 1024 and 2048, Bluestein for 43, 683 and 10923, Bluestein forced for 768, which
    neither factors into line lengths nor needs it), a band not containing 0, a band far off
    centre that folds several coefficients into each output bin, and the largest
    mixed-workload length (512 sampled points).  Odd N (683, 171, 10923) takes the full-length
    transform of each real row (Bluestein at 1536, 384 and 24576)."""
    from paper_1802_10291_amd import Plan1D
    cnt = 2 if N > 8192 else 3
    g = S.smooth_noisy_batch(70, cnt, M, N, 2 * M * N)
    chans = deriv_channels(M)
    plan = Plan1D(N=N, n_out=n_out, channels=chans, n1=n1)
    if plan.info.path == 1:
        plan.set_variant("real_two_pass")
    assert plan.variant == "real_two_pass"
    y = plan.reconstruct(torch_cuda.from_numpy(g).cuda()).cpu().numpy().astype(np.float64)
    ch = O.Channels(N=N, kinds=[O.MULT_DERIV] * M, orders=list(range(M)), n1=n1)
    if N > 8192:
        band = O.recover_band(ch, g.astype(np.float64))
        idx = np.random.default_rng(1).choice(n_out, 512, replace=False)
        for b in range(cnt):
            want = O.evaluate_band(band[b], ch.n1, 2 * np.pi * idx / n_out)
            assert rel(y[b, 0, idx], want) <= 1e-5, b
    else:
        want = O.reconstruct_1d(ch, g.astype(np.float64), n_out)
        for b in range(cnt):
            assert rel(y[b], want[b]) <= 1e-5, b


@pytest.mark.parametrize("N,n_out,M", [(1024, 4096, 2), (683, 8192, 3), (1366, 16384, 3), (512, 2048, 4)])
def test_real_two_pass_f16_storage(torch_cuda, N, n_out, M):
    """The real-mode path with FP16 samples and outputs (pairs read by the first pass, the last
    pass writes half2), derivative channels in units of N; within FP16 rounding of the oracle."""
    from paper_1802_10291_amd import Plan1D
    g = S.smooth_noisy_batch(80, 3, M, N, 2 * M * N, dtype=np.float16, deriv_scale=N)
    plan = Plan1D(N=N, n_out=n_out, channels=[("table", t) for t in scaled_deriv_tables(M, N)], storage="f16")
    plan.set_variant("real_two_pass")
    y = plan.reconstruct(torch_cuda.from_numpy(g).cuda()).cpu().numpy().astype(np.float64)
    want = oracle_1d(g, M, N, n_out, scaled=True)
    for b in range(3):
        assert rel(y[b], want[b]) <= 1e-3, b


def test_2d_variants_match_oracle(torch_cuda):
    from paper_1802_10291_amd import Plan2D
    lr = SI.random_field_images(3, 2, 64, 64)
    want = O.upsample_2d(lr.astype(np.float64), 2)
    plan = Plan2D(64, 64, 2)
    assert plan.variants() == ["multipass_r8", "line_pass"] and plan.variant == "line_pass"
    for v in plan.variants():
        plan.set_variant(v)
        hr = plan.upsample(torch_cuda.from_numpy(lr).cuda()).cpu().numpy()
        assert rel(hr, want) <= 1e-5, v


# ------------------------------------------------------------------ autotuner
def test_autotune_picks_fastest_and_caches(torch_cuda, tmp_path, monkeypatch):
    from paper_1802_10291_amd import Plan1D
    cache = str(tmp_path / "tune.json")
    plan = Plan1D(N=1366, n_out=16384, channels=deriv_channels(3))
    name, ms, cached = plan.autotune(256, cache)
    assert not cached and name in plan.variants() and plan.variant == name
    assert set(ms) == set(plan.variants()) and all(v > 0 for v in ms.values())
    assert ms[name] == min(ms.values())
    doc = json.load(open(cache))
    assert len(doc["entries"]) == 1 and doc["entries"][0]["variant"] == plan.info.variant
    name2, _, cached2 = plan.autotune(256, cache)
    assert cached2 and name2 == name
    # a second shape adds an entry; the file stays valid JSON
    other = Plan1D(N=96, n_out=1152, channels=deriv_channels(3))
    other.autotune(64, cache)
    assert len(json.load(open(cache))["entries"]) == 2
    # plans created with the cache in the environment start on the recorded variant
    monkeypatch.setenv("MCI_TUNE_CACHE", cache)
    for forced in ("multipass_r4", "fused_t1"):
        plan.set_variant(forced)
        doc = json.load(open(cache))
        for e in doc["entries"]:
            if "|N1366|" in e["key"]:
                e["variant"] = plan.info.variant
        with open(cache, "w") as f:
            f.write('{"version": 1, "entries": [\n' + ",\n".join(json.dumps(e) for e in doc["entries"]) + "\n]}\n")
        fresh = Plan1D(N=1366, n_out=16384, channels=deriv_channels(3))
        assert fresh.variant == forced


def test_autotune_2d_plan(torch_cuda, tmp_path):
    from paper_1802_10291_amd import Plan2D
    plan = Plan2D(128, 128, 2)
    name, ms, cached = plan.autotune(8, str(tmp_path / "t.json"))
    assert set(ms) == {"multipass_r8", "line_pass"} and name == min(ms, key=ms.get)


# ------------------------------------------------------------------ uneven batches
# (kind, args): 1-D (N, M, n_out) with single-pass and multi-pass classes, Bluestein and
# smooth lengths; 2-D (side, scale) with line-pass and multi-pass classes
MIX = [("1d", (1366, 3, 16384)), ("1d", (1000, 3, 16384)), ("1d", (86, 3, 1024)), ("1d", (64, 4, 1024)),
       ("1d", (128, 2, 1024)), ("2d", (64, 2)), ("2d", (48, 2)), ("2d", (40, 2))]   # 40: no line pass, multi-pass 2-D


def _mixed_batch(torch, storage="native", lanes=16, seed=0, per_class=3):
    from paper_1802_10291_amd import Batch, Plan1D, Plan2D
    np_dt = np.float16 if storage == "f16" else np.float32
    f16 = storage == "f16"
    plans, data = [], []
    for c, (kind, a) in enumerate(MIX):
        if kind == "1d":
            N, M, n_out = a
            chans = [("table", t) for t in scaled_deriv_tables(M, N)] if f16 else deriv_channels(M)
            plans.append(Plan1D(N=N, n_out=n_out, channels=chans, storage=storage))
            data.append(S.smooth_noisy_batch(100 * c, per_class, M, N, 2 * M * N, dtype=np_dt,
                                             deriv_scale=N if f16 else 1.0))
        else:
            side, s = a
            plans.append(Plan2D(side, side, s, storage=storage))
            data.append(SI.random_field_images(100 * c, per_class, side, side).astype(np_dt))
    order = [(c, k) for c in range(len(MIX)) for k in range(per_class)]
    np.random.default_rng(seed).shuffle(order)
    batch = Batch([plans[c] for c, _ in order], lanes=lanes)
    packed = np.zeros(batch.in_elems, dtype=np_dt)
    for (c, k), off in zip(order, batch.in_offsets):
        x = data[c][k].ravel()
        packed[off:off + x.size] = x
    return batch, plans, data, order, packed


def _unpack(batch, plans, order, out_host):
    res = []
    for (c, k), off in zip(order, batch.out_offsets):
        n = plans[c].instance_sizes()[1]
        res.append(out_host[off:off + n])
    return res


@pytest.mark.parametrize("storage,lanes,merged", [("native", 16, False), ("native", 4, False), ("native", 1, False),
                                                  ("f16", 16, False), ("native", 16, True), ("native", 1, True),
                                                  ("f16", 16, True)])
def test_uneven_batch_matches_single_calls_and_oracle(torch_cuda, monkeypatch, storage, lanes, merged):
    """Each class's own launches on the lanes, or (merged) persistent launches over job tables
    for the classes whose kernels record as jobs: both bit-identical to single-plan calls."""
    torch = torch_cuda
    if merged:
        monkeypatch.setenv("MCI_BATCH_MERGED", "1")
    batch, plans, data, order, packed = _mixed_batch(torch, storage, lanes)
    monkeypatch.delenv("MCI_BATCH_MERGED", raising=False)
    dev_in = torch.from_numpy(packed).cuda()
    out = torch.full((batch.out_elems,), float("nan"), dtype=dev_in.dtype, device="cuda")
    batch.run(dev_in, out)
    host = out.cpu().numpy().astype(np.float64)
    # everything outside the instances' extents is untouched
    mask = np.ones(batch.out_elems, dtype=bool)
    for (c, k), off in zip(order, batch.out_offsets):
        mask[off:off + plans[c].instance_sizes()[1]] = False
    assert np.isnan(host[mask]).all()
    # bit-identical to single-plan calls, and within tolerance of the oracle
    singles = []
    for c, (kind, a) in enumerate(MIX):
        x = torch.from_numpy(data[c]).cuda()
        y = plans[c].reconstruct(x) if kind == "1d" else plans[c].upsample(x)
        singles.append(y.cpu().numpy().astype(np.float64).reshape(len(data[c]), -1))
    tol = 1e-3 if storage == "f16" else 1e-5
    oracle_cache = {}
    for (c, k), got in zip(order, _unpack(batch, plans, order, host)):
        assert np.array_equal(got, singles[c][k]), (MIX[c], k)
        kind, a = MIX[c]
        if c not in oracle_cache:
            if kind == "1d":
                N, M, n_out = a
                oracle_cache[c] = oracle_1d(data[c], M, N, n_out, scaled=storage == "f16").reshape(len(data[c]), -1)
            else:
                oracle_cache[c] = O.upsample_2d(data[c].astype(np.float64), a[1]).reshape(len(data[c]), -1)
        assert rel(got, oracle_cache[c][k]) <= tol, (MIX[c], k)


@pytest.mark.parametrize("merged", [False, True])
def test_uneven_batch_graph_capture_replays(torch_cuda, monkeypatch, merged):
    """The whole mixed batch (16 lanes forked from and joined into the capture stream) is
    captured as one graph; each replay, with eager work and new input values in between,
    reproduces the eager result for the current input."""
    torch = torch_cuda
    if merged:
        monkeypatch.setenv("MCI_BATCH_MERGED", "1")
    batch, plans, data, order, packed = _mixed_batch(torch, "native", 16)
    monkeypatch.delenv("MCI_BATCH_MERGED", raising=False)
    dev_in = torch.from_numpy(packed).cuda()
    out = torch.zeros(batch.out_elems, dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch.run(dev_in, out)          # warm-up; allocates the workspace outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.run(dev_in, out)
    for r in range(3):
        scale = 1.0 + 0.5 * r
        dev_in.copy_(torch.from_numpy(packed).cuda() * scale)
        ref = batch.run(dev_in, torch.empty_like(out))
        torch.cuda.synchronize()
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {r}"


def test_uneven_batch_rejects_bad_layouts(torch_cuda):
    from paper_1802_10291_amd import Batch, MCIError, Plan1D, Plan2D
    p = Plan1D(N=64, n_out=512, channels=deriv_channels(2))
    q = Plan2D(32, 32, 2, storage="f16")
    n_in, n_out = p.instance_sizes()
    with pytest.raises(MCIError):       # overlapping outputs
        Batch([p, p], offsets=([0, n_in], [0, n_out - 4]))
    with pytest.raises(MCIError):       # misaligned offset
        Batch([p], offsets=([2], [0]))
    with pytest.raises(MCIError):       # mixed element types
        Batch([p, q])
    b = Batch([p, p], offsets=([0, 0], [0, n_out]))   # shared input is allowed
    assert b.in_elems == n_in and b.out_elems == 2 * n_out


@pytest.mark.parametrize("key", [("1d", 65536, 2), ("1d", 49152, 3), ("1d", 65536, 4), ("2d", 1024)])
def test_uneven_workload_largest_classes_sampled_parity(torch_cuda, key):
    """The mixed workload's largest classes at full size, in one batch with a small class:
    1-D outputs checked at 512 sampled grid points each (relative L2 and element-wise over the
    sample) against the oracle's recovered band evaluated there directly; 2-D images against
    the full oracle."""
    from paper_1802_10291_amd import Batch, Plan1D, Plan2D
    torch = torch_cuda
    pool = U.class_pool(key, 99, 2)
    if key[0] == "1d":
        _, L, M = key
        N = -(-L // M)
        plan = Plan1D(N=N, n_out=4 * L, channels=deriv_channels(M))
    else:
        plan = Plan2D(key[1] // 2, key[1] // 2, 2)
    small = Plan1D(N=64, n_out=1024, channels=deriv_channels(2))
    small_in = S.smooth_noisy_batch(0, 1, 2, 64, 256)
    batch = Batch([plan, small, plan])
    packed = np.zeros(batch.in_elems, dtype=np.float32)
    for x, off in zip([pool[0], small_in[0], pool[1]], batch.in_offsets):
        packed[off:off + x.size] = x.ravel()
    out = batch.run(torch.from_numpy(packed).cuda()).cpu().numpy().astype(np.float64)
    n_out_elems = plan.instance_sizes()[1]
    got = [out[batch.out_offsets[i]:batch.out_offsets[i] + n_out_elems] for i in (0, 2)]
    if key[0] == "1d":
        ch = O.Channels(N=N, kinds=[O.MULT_DERIV] * M, orders=list(range(M)))
        band = O.recover_band(ch, pool.astype(np.float64))
        idx = np.random.default_rng(L + M).choice(4 * L, 512, replace=False)
        for b in range(2):
            want = O.evaluate_band(band[b], ch.n1, 2 * np.pi * idx / (4 * L))
            assert rel(got[b][idx], want) <= 1e-5
    else:
        want = O.upsample_2d(pool.astype(np.float64), 2)
        for b in range(2):
            assert rel(got[b], want[b].ravel()) <= 1e-5
    small_want = oracle_1d(small_in, 2, 64, 1024)[0, 0]
    assert rel(out[batch.out_offsets[1]:batch.out_offsets[1] + 1024], small_want) <= 1e-5


def test_kernel_names_follow_the_variant(torch_cuda):
    """mci_plan_kernel_name describes the active variant's kernels."""
    from paper_1802_10291_amd import Plan1D, Plan2D
    plan = Plan1D(N=1366, n_out=16384, channels=deriv_channels(3))
    assert plan.kernel_name().startswith("k_mci1d_fused: forward split-Bluestein 1024-point, output 2 x 4096-point")
    plan.set_variant("real_two_pass")
    assert plan.kernel_name().startswith("real two-pass: k_fft_lines forward")
    plan.set_variant("multipass_r4")
    assert plan.kernel_name().startswith("multi-pass radix-4 passes")
    assert Plan2D(128, 128, 2).kernel_name().startswith("k_line_pass: columns 128 -> rows 128, scale 2")
