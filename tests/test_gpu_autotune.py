"""EM launch plans: every launch variant of every bucket reproduces the
oracle's replayed sweeps (the autotuner may pick any of them), and the
autotuner installs a plan that keeps the compress results within the same
bars."""
import numpy as np
import pytest

import oracle
from paper_2007_12273_amd import synth

from gpu_util import dev, host, to_gpu, torch
import fp32_parity

pytestmark = pytest.mark.gpu

MAXN16 = [128, 256, 512, 768, 1024, 1280, 1536, 1792, 2048, 2560, 4096, 8192]
MAXN8 = [64, 128, 256, 512, 1024, 1536, 2048, 2560, 3072, 3584, 4096, 8192]
# (particles per thread, register-resident densities, lean build)
VARIANTS = [(1, True, False), (2, True, False), (4, True, False), (8, True, False), (8, False, False),
            (16, False, False), (1, True, True), (2, True, True), (4, False, True), (8, False, True),
            (5, True, False), (6, True, False), (7, True, False)]


def _codes(kmax, variant, D=3):
    P, se, lean = variant
    if se and 5 <= P <= 7 and kmax <= 8:
        return None
    out = []
    for m in (MAXN8 if kmax <= 8 else MAXN16):
        w = -(-m // (64 * P))
        if w > (16 if lean else 8):
            out.append(None)
        else:
            out.append(P * 1000 + w * 10 + (1 if se else 0) + (2 if lean else 0))
    return out


def _batch(D=3):
    sizes = [40, 64, 100, 128, 200, 256, 400, 512, 700, 768, 900, 1024, 1200, 1280, 1500, 1536, 1700, 1792, 1900,
             2048, 2500, 3000, 3584, 4096, 5000]
    parts = [synth.random_cells(300 + i, 1, D, n, n, k_lo=2, k_hi=4) for i, n in enumerate(sizes)]
    return synth.concat_cells(parts)


@pytest.mark.parametrize("D,kmax", [(3, 8), (3, 16), (1, 8), (1, 16)])
def test_every_variant_matches_oracle_replay(D, kmax):
    from paper_2007_12273_amd import api
    d = _batch(D)
    v, a, off = to_gpu(d)
    o = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=kmax, seed=9, max_sweeps=20)
    fs = torch.from_numpy(o["sweeps"].astype(np.int32)).to(dev())
    res = fp32_parity.resolution(d, kmax, 9, o["sweeps"], o)
    default = (MAXN8 if kmax <= 8 else MAXN16)
    try:
        for var in VARIANTS:
            codes = _codes(kmax, var, D)
            if codes is None:
                continue
            # buckets the variant cannot cover run recomputed densities with
            # 16 particles per thread
            fill = [c if c is not None else 16000 + 10 * (-(-default[b] // 1024)) for b, c in enumerate(codes)]
            api.autotune_set(D, kmax, fill)
            g = host(api.compress(v, a, off, kmax, seed=9, fixed_sweeps=fs, max_sweeps=20))
            assert np.array_equal(g["sweeps"], o["sweeps"])
            fp32_parity.check(g, o, d, res, "D %d variant %s kmax %d" % (D, var, kmax))
    finally:
        api.autotune_reset()


def test_autotune_installs_a_working_plan():
    from paper_2007_12273_amd import api
    d = synth.make("weibel_3v")
    off = d["cell_off"]
    nc = 512
    sub = dict(v=d["v"][:off[nc]], alpha=d["alpha"][:off[nc]], cell_off=off[:nc + 1], D=3)
    v, a, offg = to_gpu(sub)
    comp = api.Compressor(nc, 3, 16, device=dev(), seed=2003)
    try:
        rep = comp.autotune(v, a, offg)
        print("autotune:", rep)
        assert rep["builtin_em_ms"] > 0 and rep["tuned_em_ms"] > 0
        for code, lane in zip(rep["variant"], rep["lane"]):
            assert code // 1000 in (1, 2, 4, 5, 6, 7, 8, 16) and code % 10 <= 3 and 0 <= lane <= 11
        # FP32 at kmax 16: the cells of 2049-2560 and 2561-4096 particles run
        # eight waves of 5 and 8 register-resident particles or a lean build of
        # more than 8 waves, those of 4097-8192 particles the 16-wave lean
        # build of 8 recomputed particles
        assert rep["variant"][9] in (5081, 4102), rep["variant"]
        assert rep["variant"][10] in (8081, 4162) and rep["variant"][11] == 8162, rep["variant"]
        # the installed plan (tuned or the kept built-in one) is the reported one
        inst = api.autotune_get(3, 16)
        assert inst["tuned"] and inst["variant"] == list(rep["variant"]) and inst["lane"] == list(rep["lane"]), inst
        tuned = host(comp.out.as_dict())
        again = host(comp(v, a, offg).as_dict())
        for k in ("K", "sweeps", "status"):
            assert np.array_equal(tuned[k], again[k]), k
        o = oracle.compress(sub["v"], sub["alpha"], sub["cell_off"], kmax=16, seed=2003, max_sweeps=60)
        fs = torch.from_numpy(o["sweeps"].astype(np.int32)).to(dev())
        g = host(comp(v, a, offg, fixed_sweeps=fs).as_dict())
        res = fp32_parity.resolution(sub, 16, 2003, o["sweeps"], o)
        fp32_parity.check(g, o, sub, res, "tuned plan replay")
    finally:
        api.autotune_reset()


def test_plan_file_round_trip(tmp_path):
    """A plan written by gm_autotune_save and read back by gm_autotune_load
    after a reset is the same plan (variants, streams, launch order) and
    gives bit-identical compress results; lines of another device are
    skipped and kept by a later save; a file with an invalid line installs
    nothing."""
    from paper_2007_12273_amd import api
    d = synth.make("weibel_3v")
    off = d["cell_off"]
    nc = 256
    sub = dict(v=d["v"][:off[nc]], alpha=d["alpha"][:off[nc]], cell_off=off[:nc + 1], D=3)
    v, a, offg = to_gpu(sub)
    comp = api.Compressor(nc, 3, 16, device=dev(), seed=2003)
    path = tmp_path / "plans.txt"
    codes = [2011, 4011, 4021, 4031, 8021, 5041, 6041, 7041, 4081, 5081, 8081, 8162]
    lanes = [11 - b for b in range(12)]
    order = [5, 4, 3, 2, 1, 0, 11, 10, 9, 8, 7, 6]
    try:
        api.autotune_reset()
        assert not api.autotune_get(3, 16)["tuned"]
        api.autotune_set(3, 16, codes, lanes)
        ref = host(comp(v, a, offg).as_dict())
        other = "gmcr-plan 1 gfx000 7 3 16 0 0 " + " ".join(["16080"] * 12 + ["0"] * 12 + [str(b) for b in range(12)])
        path.write_text("# plans\n" + other + "\n")
        api.autotune_save(path)
        lines = path.read_text().splitlines()
        assert other in lines and len(lines) == 2, lines
        mine = [l for l in lines if l != other][0].split()
        assert [int(x) for x in mine[8:20]] == codes and [int(x) for x in mine[20:32]] == lanes, mine
        mine[32:44] = [str(x) for x in order]
        text = "\n".join([other, " ".join(mine)]) + "\n"
        path.write_text(text)
        api.autotune_reset()
        assert not api.autotune_get(3, 16)["tuned"]
        assert api.autotune_load(path) == 1
        loaded = api.autotune_get(3, 16)
        assert loaded == {"variant": codes, "lane": lanes, "order": order, "tuned": True}, loaded
        again = host(comp(v, a, offg).as_dict())
        for k in ("K", "sweeps", "visits", "status", "L_pen", "omega", "mu", "sigma"):
            assert np.array_equal(again[k], ref[k]), k
        # an invalid line (a variant that does not cover its bucket, an order
        # that is not a permutation) rejects the whole file
        for bad in (" ".join(mine[:19] + ["4081"] + mine[20:]), " ".join(mine[:43] + ["5"])):
            api.autotune_reset()
            bad_path = tmp_path / "bad.txt"
            bad_path.write_text(other + "\n" + bad + "\n")
            with pytest.raises(RuntimeError):
                api.autotune_load(bad_path)
            assert not api.autotune_get(3, 16)["tuned"]
    finally:
        api.autotune_reset()


@pytest.mark.parametrize("which", ["weibel", "no_large_cells"])
def test_two_step_release_leaves_results_unchanged(which):
    """The EM launches of the buckets whose workgroups fill a CU are released
    before the others (with a short device-side wait between); a plan with
    the same variants whose CU-filling buckets sit on the caller's stream
    releases everything at once.  Each cell is fitted by the same variant
    either way, so the two records are bit-identical: with the large-cell
    buckets populated (Weibel-like cells of up to 5000 particles) and empty
    (the wait then ends at once)."""
    from paper_2007_12273_amd import api
    d = synth.make("weibel_3v")
    off = d["cell_off"]
    n = np.diff(off)
    if which == "weibel":
        cells = np.arange(768)
    else:
        cells = np.flatnonzero(n <= 1792)[:768]
    parts = [dict(v=d["v"][off[c]:off[c + 1]], alpha=d["alpha"][off[c]:off[c + 1]],
                  cell_off=np.array([0, n[c]], dtype=np.int64), D=3) for c in cells]
    sub = synth.concat_cells(parts)
    sizes = np.diff(sub["cell_off"])
    assert (sizes > 1792).any() == (which == "weibel")
    v, a, offg = to_gpu(sub)
    try:
        api.autotune_reset()
        plan = api.autotune_get(3, 16)
        codes = plan["variant"]
        # waves of each code; 8+ (16+ for lean builds) fill a CU
        fills = [(c // 10) % 100 >= (16 if c % 10 & 2 else 8) for c in codes]
        assert any(fills) and not all(fills), codes
        staged = host(api.compress(v, a, offg, 16, seed=31))
        api.autotune_set(3, 16, codes, [12 if f else b for b, f in enumerate(fills)])
        together = host(api.compress(v, a, offg, 16, seed=31))
        for k in staged:
            assert np.array_equal(staged[k], together[k], equal_nan=True), k
        assert (staged["K"] > 0).all()
    finally:
        api.autotune_reset()
