"""GPU tests of the ragged batched path (nslct_batch_*): every image of a
batch with its own matrix and size, against the FP64 oracle (element by
element) and the per-image launch loop (to rounding: the batch and the
single-image passes may split a line over threads differently); every
schedule of one line plan gives the same bits; graph replays interleaved
with other work."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import chain, plan as oplan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def nl(torch):
    import paper_1707_03688_amd as _nl
    return _nl


def _batch(nl, sizes, seed, precision="c64", rect=False):
    cands = synth.symplectic_candidates(seed)
    plans, oplans = [], []
    for i, s in enumerate(sizes):
        M = next(cands)
        Nx, Ny = (s, sizes[(i + 1) % len(sizes)]) if rect else (s, s)
        d = (2 * np.pi / max(Nx, Ny)) ** 0.5
        po = oplan.plan(M, Nx, Ny, d, d)
        plans.append(nl.Plan.from_stages(po.typ, po.mats, Nx, Ny, d, d, precision))
        oplans.append(po)
    return nl.Batch(plans), oplans


TPL = {0: {64: 8, 128: 16, 192: 8, 256: 16, 384: 16, 512: 64, 768: 32, 1024: 64},
       1: {64: 16, 128: 8, 192: 16, 256: 32, 384: 32, 512: 32, 768: 64, 1024: 32}}


def _plan0(b, skip=()):
    """Every native group on line plan 0 (the single-image kernels' split of
    a line), 256 threads per work item, its tuned grid."""
    for (col, N), sch in b.schedules().items():
        if N not in skip:
            b.set_group(col, N, 256 // TPL[0][N], sch["mult"], plan=0)


def _rel(a, b):
    return ((a - b).abs().pow(2).sum() / b.abs().pow(2).sum()).sqrt().item()


@pytest.mark.parametrize("rect", [False, True])
def test_batched_matches_loop_bitwise_and_oracle(torch, nl, rect):
    """The tuned batch against the FP64 oracle (every image) and the
    per-image loop (to rounding); graph replay and plain launches give the
    same bits."""
    sizes = [64, 384, 128, 768, 256, 192, 512, 64, 128, 384, 1024]
    b, oplans = _batch(nl, sizes, seed=31, rect=rect)
    g = synth.complex_normal((b.total,), seed=2)
    x = torch.from_numpy(g).to(torch.complex64).cuda()
    out_graph = b.forward(x)
    out_plain = b.run(x, mode=1)
    out_loop = b.run(x, mode=2)
    torch.cuda.synchronize()
    assert torch.equal(out_graph, out_plain)
    assert _rel(out_graph, out_loop) <= 1e-6
    got = out_graph.cpu().numpy()
    for o, p, po in zip(b.offsets, b.plans, oplans):  # every image, 64^2 to 1024^2
        gi = g[o:o + p.Nx * p.Ny].reshape(p.Nx, p.Ny)
        ref = chain.forward(po, gi)
        assert chain.rel_l2(got[o:o + p.Nx * p.Ny].reshape(p.Nx, p.Ny), ref) <= 1e-5
    back = b.inverse(out_graph).cpu().numpy()
    assert chain.rel_l2(back, g) <= 1e-5


def test_paired_rectangular_batch(torch, nl):
    """Rectangular images whose row and column line lengths pair up (every
    image with Ny = 256 has Nx = 512, and so on; a Bluestein length among
    them): the batch runs each pair's passes as one independent sequence.
    Against the oracle (every image), the per-image loop (to rounding), graph
    and plain launches bitwise, and the inverse."""
    shapes = [(512, 256), (128, 384), (512, 256), (64, 64), (128, 384), (768, 100), (512, 256)]
    cands = synth.symplectic_candidates(34)
    plans, oplans = [], []
    for Nx, Ny in shapes:
        d = (2 * np.pi / max(Nx, Ny)) ** 0.5
        po = oplan.plan(next(cands), Nx, Ny, d, d)
        plans.append(nl.Plan.from_stages(po.typ, po.mats, Nx, Ny, d, d, "c64"))
        oplans.append(po)
    b = nl.Batch(plans)
    g = synth.complex_normal((b.total,), seed=6)
    x = torch.from_numpy(g).to(torch.complex64).cuda()
    out_graph = b.forward(x)
    out_plain = b.run(x, mode=1)
    out_loop = b.run(x, mode=2)
    torch.cuda.synchronize()
    assert torch.equal(out_graph, out_plain)
    assert _rel(out_graph, out_loop) <= 1e-6
    got = out_graph.cpu().numpy()
    for o, p, po in zip(b.offsets, b.plans, oplans):
        ref = chain.forward(po, g[o:o + p.Nx * p.Ny].reshape(p.Nx, p.Ny))
        assert chain.rel_l2(got[o:o + p.Nx * p.Ny].reshape(p.Nx, p.Ny), ref) <= 1e-5
    back = b.inverse(out_graph).cpu().numpy()
    assert chain.rel_l2(back, g) <= 1e-5


def test_graph_replays_are_stable(torch, nl):
    """Repeated graph replays with unrelated eager work between them all equal
    the eager (non-graph) result; in-place replays too."""
    b, _ = _batch(nl, [256, 128, 384, 64], seed=32)
    x = torch.from_numpy(synth.complex_normal((b.total,), seed=3)).to(torch.complex64).cuda()
    ref = b.run(x, mode=1)
    out = torch.empty_like(x)
    for k in range(4):
        b.forward(x, out=out)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {k}"
        del junk
    y = x.clone()
    b.forward(y, out=y)
    assert torch.equal(y, ref)


def test_batched_c128(torch, nl):
    b, oplans = _batch(nl, [64, 96 * 2, 128], seed=33, precision="c128")
    g = synth.complex_normal((b.total,), seed=4)
    x = torch.from_numpy(g).cuda()
    got = b.forward(x).cpu().numpy()
    for o, p, po in zip(b.offsets, b.plans, oplans):
        ref = chain.forward(po, g[o:o + p.Nx * p.Ny].reshape(p.Nx, p.Ny))
        assert chain.rel_l2(got[o:o + p.Nx * p.Ny].reshape(p.Nx, p.Ny), ref) <= 1e-11


@pytest.mark.skip(reason="batches take native sides 64..1024 only: a build that added every native side "
                         "from 2 to 2048 passed this test, but a later batch test in the same process then "
                         "ended in a host segmentation fault whose cause was not found, so that build was "
                         "withdrawn")
@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_every_native_side_in_a_batch(torch, nl, precision):
    """Native sides from 2 to 2048 (2^k and 3 * 2^k) batch together:
    rectangular images pairing short and long sides, every image against the
    FP64 oracle, graph and plain launches bitwise, the per-image loop to
    rounding, and the inverse."""
    shapes = [(2, 2048), (2048, 4), (6, 12), (8, 24), (16, 48), (32, 96), (12, 2), (24, 8), (48, 32),
              (96, 16), (4, 6), (64, 2048)]
    cands = synth.symplectic_candidates(53)
    plans, oplans = [], []
    for Nx, Ny in shapes:
        d = (2 * np.pi / max(Nx, Ny)) ** 0.5
        po = oplan.plan(next(cands), Nx, Ny, d, d)
        plans.append(nl.Plan.from_stages(po.typ, po.mats, Nx, Ny, d, d, precision))
        oplans.append(po)
    b = nl.Batch(plans)
    g = synth.complex_normal((b.total,), seed=9)
    dt = torch.complex64 if precision == "c64" else torch.complex128
    tol = 1e-5 if precision == "c64" else 1e-11
    x = torch.from_numpy(g).to(dt).cuda()
    out = b.forward(x)
    assert torch.equal(out, b.run(x, mode=1))
    assert _rel(out, b.run(x, mode=2)) <= (1e-6 if precision == "c64" else 1e-13)
    got = out.cpu().numpy()
    for o, p, po in zip(b.offsets, b.plans, oplans):
        ref = chain.forward(po, g[o:o + p.Nx * p.Ny].reshape(p.Nx, p.Ny))
        assert chain.rel_l2(got[o:o + p.Nx * p.Ny].reshape(p.Nx, p.Ny), ref) <= tol, (p.Nx, p.Ny)
    assert chain.rel_l2(b.inverse(out).cpu().numpy(), g) <= tol


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_bluestein_sizes_in_a_batch(torch, nl, precision):
    """Sides without a native line plan (Bluestein line DFTs) batch with the
    native ones: every image against the FP64 oracle, the graph replay
    against the per-image loop bitwise (same Bluestein code), inverse round
    trip; the zero-padding sizes 165 + dN of the accuracy sweep in one batch."""
    sizes = [100, 165, 175, 64, 185, 257, 128, 300]
    b, oplans = _batch(nl, sizes, seed=51, precision=precision, rect=True)
    g = synth.complex_normal((b.total,), seed=8)
    dt = torch.complex64 if precision == "c64" else torch.complex128
    tol = 1e-5 if precision == "c64" else 1e-11
    x = torch.from_numpy(g).to(dt).cuda()
    out = b.forward(x)
    got = out.cpu().numpy()
    for o, p, po in zip(b.offsets, b.plans, oplans):
        ref = chain.forward(po, g[o:o + p.Nx * p.Ny].reshape(p.Nx, p.Ny))
        assert chain.rel_l2(got[o:o + p.Nx * p.Ny].reshape(p.Nx, p.Ny), ref) <= tol, (p.Nx, p.Ny)
    sch = b.schedules()
    for N in (100, 165, 175, 185, 257, 300):
        assert sch[(1, N)]["plan"] == 0
    _plan0(b, skip=(100, 165, 175, 185, 257, 300))
    if precision == "c128":  # the single-image passes split 64-long complex128 lines the other way
        for (col, N), sch in b.schedules().items():
            if N == 64:
                b.set_group(col, N, 256 // TPL[1][N], sch["mult"], plan=1)
    assert torch.equal(b.forward(x), b.run(x, mode=2))
    back = b.inverse(out).cpu().numpy()
    assert chain.rel_l2(back, g) <= tol


def test_batch_rejects_bad_input(torch, nl):
    M = next(synth.symplectic_candidates(1))
    with pytest.raises(nl.NslctError):
        nl.Batch([nl.Plan(M, 2048, 2048)])
    with pytest.raises(nl.NslctError):  # native, but not a batched line length
        nl.Batch([nl.Plan(M, 48, 64)])
    with pytest.raises(nl.NslctError):
        nl.Batch([nl.Plan(M, 64, 64), nl.Plan(M, 64, 64, precision="c128")])


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_every_grid_mode_gives_the_same_bits(torch, nl, precision):
    """The persistent grids (1, 2, 4, 8 workgroups per CU: the looping
    kernel) and one workgroup per item (the loop-free kernel) compute every
    item with the same code: graph replays in each mode give the same bits,
    forward and inverse, for complex64 (wide column tiles) and complex128,
    and match the per-image loop to rounding; invalid modes are rejected."""
    sizes = [1024, 768, 64, 384, 512, 128, 256, 192]
    b, _ = _batch(nl, sizes, seed=47, precision=precision)
    _plan0(b)
    g = synth.complex_normal((b.total,), seed=5)
    x = torch.from_numpy(g).to(torch.complex64 if precision == "c64" else torch.complex128).cuda()
    tol = 1e-6 if precision == "c64" else 1e-13
    ref_f = b.run(x, mode=1)
    ref_i = b.run(x, direction=1, mode=1)
    assert _rel(ref_f, b.run(x, mode=2)) <= tol and _rel(ref_i, b.run(x, direction=1, mode=2)) <= tol
    for mult in (0, 1, 2, 4, 8):
        b.set_grid(mult)
        assert torch.equal(b.forward(x), ref_f), mult
        assert torch.equal(b.inverse(x), ref_i), mult
        assert torch.equal(b.run(x, mode=1), ref_f), mult
    for bad in (3, -1, 16):
        with pytest.raises(nl.NslctError):
            b.set_grid(bad)



@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_every_schedule_candidate(torch, nl, precision):
    """Each group's candidates — line plan 0 or 1 (another split of the line
    over threads and radices) and tile width (lines per work item for 256,
    512 or 1024 threads, as LDS allows): the widths of one plan give the same
    bits, and every candidate the per-image loop's result to rounding."""
    sizes = [1024, 768, 64, 384, 512, 128, 256, 192]
    b, _ = _batch(nl, sizes, seed=48, precision=precision)
    g = synth.complex_normal((b.total,), seed=6)
    x = torch.from_numpy(g).to(torch.complex64 if precision == "c64" else torch.complex128).cuda()
    ref = b.run(x, mode=2)
    tol = 1e-6 if precision == "c64" else 1e-13
    tuned = b.schedules()
    _plan0(b)
    for (col, N), sch in tuned.items():
        for plan in (0, 1):
            first, tried = None, 0
            for threads in (256, 512, 1024):
                lines = threads // TPL[plan][N]
                try:
                    b.set_group(col, N, lines, 2, plan=plan)
                except nl.NslctError:
                    continue  # not a candidate (LDS, or 1024 threads on a row pass)
                tried += 1
                out = b.forward(x)
                assert b.group(col, N)["plan"] == plan and b.group(col, N)["lines"] == lines
                assert _rel(out, ref) <= tol, (col, N, plan, lines)
                if first is None:
                    first = out
                assert torch.equal(out, first), (col, N, plan, lines)
            assert tried >= 1, (col, N, plan)
            b.set_group(col, N, 256 // TPL[0][N], sch["mult"], plan=0)
    with pytest.raises(nl.NslctError):
        b.set_group(0, 1024, 4, 2, plan=2)
    for (col, N), sch in tuned.items():
        b.set_group(col, N, sch["lines"], sch["mult"], plan=sch["plan"])
    assert _rel(b.forward(x), ref) <= tol


def test_schedule_cache(torch, nl, tmp_path, monkeypatch):
    """The first batch of a shape tunes its groups and writes the schedule
    cache; the same batch built again takes every schedule from it (no
    tuning run) and gives the same bits."""
    monkeypatch.setenv("NSLCT_TUNE_CACHE", str(tmp_path / "sched.txt"))
    b1, _ = _batch(nl, [512, 128, 256, 128], seed=49)
    s1 = b1.schedules()
    assert not any(v["cached"] for v in s1.values()) and b1.tuned_us > 0
    lines = (tmp_path / "sched.txt").read_text().splitlines()
    assert len(lines) == len(s1) and all(l.split()[0].startswith("gfx") and len(l.split()) == 9 for l in lines)
    b2, _ = _batch(nl, [512, 128, 256, 128], seed=49)
    s2 = b2.schedules()
    assert all(v["cached"] for v in s2.values()) and b2.tuned_us == 0
    key = lambda s: {k: (v["plan"], v["lines"], v["mult"]) for k, v in s.items()}
    assert key(s1) == key(s2)
    x = torch.from_numpy(synth.complex_normal((b1.total,), seed=7)).to(torch.complex64).cuda()
    assert torch.equal(b1.forward(x), b2.forward(x))
