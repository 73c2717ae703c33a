"""Mixed-length persistent plans and the autotuner on the GPU."""
import numpy as np
import pytest

import oracle
from gpu_util import np_dtype, rel_l2, say, tol_for
from paper_2207_06803_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_06803_amd import fftc  # noqa: E402


def pack(xs, dtype):
    return np.concatenate([x.reshape(-1) for x in xs]).astype(np_dtype(dtype))


def check_mixed_output(lengths, x_flat, y_flat, direction, dtype):
    offs = np.concatenate([[0], np.cumsum(lengths)])
    lengths = np.asarray(lengths)
    for n in np.unique(lengths):
        idx = np.nonzero(lengths == n)[0]
        xs = np.stack([x_flat[offs[i]:offs[i] + n] for i in idx])
        ys = np.stack([y_flat[offs[i]:offs[i] + n] for i in idx])
        err = rel_l2(ys, oracle.dft(xs, direction))
        assert err.max() <= tol_for(n, dtype), (n, err.max())


def run(plan, x_np):
    x = torch.from_numpy(x_np).to("cuda")
    y = torch.empty_like(x)
    plan.execute(x, y)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def test_uneven_batch_10000_full_oracle():
    # 10,000 complex64 transforms, lengths drawn uniformly over the 37-member
    # set (powers of two 8..4096 and 3, 5, 7 times powers of two up to 3584)
    g = synth.rng(2)
    lengths = synth.draw_mixed_sizes(g, 10000)
    x = synth.uniform_complex(g, (int(lengths.sum()),), np.complex64)
    say("mixed 10000 transforms, elements", int(lengths.sum()))
    with fftc.plan_mixed(lengths, fftc.FORWARD, "c64") as p:
        d = p.describe()
        assert d["variant"] == "mixed_persistent" and d["mixed_transforms"] == 10000
        assert d["mixed_classes"] == len(np.unique(lengths))
        y = run(p, x)
        y2 = run(p, x)
    assert np.array_equal(y.view(np.uint32), y2.view(np.uint32))
    check_mixed_output(lengths, x, y, fftc.FORWARD, "c64")


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("direction", [fftc.FORWARD, fftc.INVERSE])
def test_mixed_small_list(dtype, direction):
    g = synth.rng(96, 0 if dtype == "c64" else 1, direction + 1)
    lengths = np.r_[synth.draw_mixed_sizes(g, 300), [1, 2, 3, 4, 5, 7, 9, 4096, 1, 16]]
    x = synth.uniform_complex(g, (int(lengths.sum()),), np_dtype(dtype))
    with fftc.plan_mixed(lengths, direction, dtype) as p:
        y = run(p, x)
    check_mixed_output(lengths, x, y, direction, dtype)


def test_mixed_equals_per_length_plans():
    g = synth.rng(97)
    lengths = synth.draw_mixed_sizes(g, 500)
    x = synth.uniform_complex(g, (int(lengths.sum()),), np.complex64)
    with fftc.plan_mixed(lengths) as p:
        y = run(p, x)
    offs = np.concatenate([[0], np.cumsum(lengths)])
    for n in np.unique(lengths):
        idx = np.nonzero(lengths == n)[0]
        xs = np.stack([x[offs[i]:offs[i] + n] for i in idx])
        with fftc.Plan(int(n), len(idx)) as q:
            xd = torch.from_numpy(xs).to("cuda")
            yd = torch.empty_like(xd)
            q.execute(xd, yd)
            torch.cuda.synchronize()
        ys = np.stack([y[offs[i]:offs[i] + n] for i in idx])
        # same algorithm and twiddles; allow last-bit differences from code
        # generation (fused multiply-adds)
        assert rel_l2(ys, yd.cpu().numpy()).max() <= 1e-6, n


def test_direct_launch_matches_graph_replay():
    # the same kernel launched on the stream instead of replayed from the
    # plan's graph: bit-identical outputs, also across pointer changes and a
    # switch back to the graph (whose pointer arguments must follow)
    g = synth.rng(97)
    lengths = synth.draw_mixed_sizes(g, 1500)
    tot = int(lengths.sum())
    xa = torch.from_numpy(synth.uniform_complex(g, (tot,), np.complex64)).to("cuda")
    xb = torch.from_numpy(synth.uniform_complex(g, (tot,), np.complex64)).to("cuda")
    with fftc.plan_mixed(lengths, fftc.INVERSE) as p:
        ya, yb = torch.empty_like(xa), torch.empty_like(xb)
        p.execute(xa, ya)
        p.execute(xb, yb)
        torch.cuda.synchronize()
        ref_a, ref_b = ya.cpu().numpy(), yb.cpu().numpy()
        p.set_mixed_launch(fftc.MIXED_LAUNCH_DIRECT)
        for rep in range(3):
            ya.zero_(), yb.zero_()
            p.execute(xb, yb)
            p.execute(xa, ya)
            torch.cuda.synchronize()
            assert np.array_equal(ya.cpu().numpy(), ref_a) and np.array_equal(yb.cpu().numpy(), ref_b), rep
        p.set_mixed_launch(fftc.MIXED_LAUNCH_GRAPH)
        # the graph's parameters were last set for (xb, yb); the last direct
        # launch used (xa, ya), so this replay must update them
        ya.zero_(), yb.zero_()
        p.execute(xa, ya)
        torch.cuda.synchronize()
        assert np.array_equal(ya.cpu().numpy(), ref_a) and not yb.cpu().numpy().any()
        with pytest.raises(fftc.FFTCError):
            p.set_mixed_launch(7)
    with fftc.Plan(64, 4) as q:
        with pytest.raises(fftc.FFTCError):
            q.set_mixed_launch(fftc.MIXED_LAUNCH_DIRECT)  # not a mixed plan


def test_graph_replays_and_pointer_changes():
    g = synth.rng(98)
    lengths = synth.draw_mixed_sizes(g, 2000)
    tot = int(lengths.sum())
    xa = synth.uniform_complex(g, (tot,), np.complex64)
    xb = synth.uniform_complex(g, (tot,), np.complex64)
    with fftc.plan_mixed(lengths) as p:
        da, db = torch.from_numpy(xa).to("cuda"), torch.from_numpy(xb).to("cuda")
        ya, yb = torch.empty_like(da), torch.empty_like(db)
        p.execute(da, ya)
        torch.cuda.synchronize()
        ref_a = ya.cpu().numpy()
        for rep in range(4):
            # eager work and synchronisation between replays
            scratch = (da * 2).sum()
            torch.cuda.synchronize()
            yb.zero_()
            p.execute(db, yb)      # pointer change -> graph parameters updated
            ya.zero_()
            p.execute(da, ya)      # and back
            torch.cuda.synchronize()
            assert np.array_equal(ya.cpu().numpy(), ref_a), rep
            del scratch
        check_mixed_output(lengths, xb, yb.cpu().numpy(), fftc.FORWARD, "c64")


def test_autotune_records_choice():
    fftc.tune_clear()
    try:
        for n in (1024, 3584, 64):
            rs, us = fftc.autotune(n, (1 << 20) // n, "c64", reps=5)
            say(f"autotune n={n} -> {rs} {us:.2f} us")
            assert int(np.prod(rs)) == n and us > 0
            assert fftc.factorize(n)[0] == rs
            with fftc.Plan(n, 8) as p:
                assert p.describe()["radices"] == rs
    finally:
        fftc.tune_clear()


@pytest.mark.parametrize("n,dtype", [(32768, "c64"), (16384, "c128")])
def test_autotune_wide_length_times_its_compiled_lists(n, dtype):
    # past fftc_max_single_n the autotuner times the compiled wide lists only;
    # its pick is recorded and later plans run it as one kernel
    wide = [list(rs) for m, rs in fftc.compiled_lists(dtype) if m == n]
    fftc.tune_clear()
    try:
        rs, us = fftc.autotune(n, 4, dtype, reps=5)
        say(f"autotune n={n} {dtype} -> {rs} {us:.2f} us")
        assert rs in wide and us > 0
        assert fftc.factorize(n, dtype)[0] == rs
        with fftc.Plan(n, 2, fftc.FORWARD, dtype) as p:
            d = p.describe()
            assert d["radices"] == rs and d["variant"] == "single_specialised", d
    finally:
        fftc.tune_clear()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_every_compiled_body_in_a_mixed_plan(dtype, tmp_path):
    # every compiled list of the mixed lengths (N <= 4096) runs as a body of
    # the persistent kernel: round k records the k-th compiled list of each
    # length in the tuning database, plans a mixed list of those lengths (a
    # ragged count of each) and checks it against the oracle
    by_n = {}
    for n, rs in fftc.compiled_lists(dtype):
        if 2 <= n <= 4096:
            by_n.setdefault(n, []).append(rs)
    rounds = max(len(v) for v in by_n.values())
    key = fftc.tune_key()
    saved = str(tmp_path / "saved.tune")
    fftc.tune_save(saved)
    try:
        for k in range(rounds):
            ns = sorted(n for n, v in by_n.items() if k < len(v))
            db = tmp_path / f"round{k}.tune"
            db.write_text("".join(f"{key} {dtype} {n} {','.join(map(str, by_n[n][k]))} 1.0\n" for n in ns))
            fftc.tune_clear()
            assert fftc.tune_load(str(db)) == len(ns)
            lengths = np.array([n for i, n in enumerate(ns) for _ in range(1 + (i + k) % 3)], dtype=np.int64)
            g = synth.rng(150, k, 1 if dtype == "c128" else 0)
            x = synth.uniform_complex(g, (int(lengths.sum()),), np_dtype(dtype))
            d = fftc.FORWARD if k % 2 == 0 else fftc.INVERSE
            say(f"mixed bodies round {k}: {len(ns)} lengths, {len(lengths)} transforms, {dtype}, dir {d}")
            with fftc.plan_mixed(lengths, d, dtype) as p:
                y = run(p, x)
            check_mixed_output(lengths, x, y, d, dtype)
    finally:
        fftc.tune_clear()
        fftc.tune_load(saved)
