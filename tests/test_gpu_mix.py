"""The second-pass baselines of the learned proposal on the GPU: the density
g(j) + mix mean g (pass2_mix; 0 is Sec. 5's g, +inf the uniform density)
against the oracle's weights_from_g, bit-exact in the kernel's precision (the
FP32 column statistics), and the second pass drawn from those weights
bit-exact, on every slice of the tiny workload (64x64 points, 16 slices of
256 rows, 1,024 singleton clusters, 5% + 5%), and on the mid workload's
slices (512x512 points, 256 columns per slice) at 5% for one mix."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from _gpu_common import keys_to_ij, log, run_frame  # noqa: E402
from oracle.sampling import pass2, weights_from_g  # noqa: E402
from paper_2202_12567_amd import api  # noqa: E402
from scenegen import make_scene  # noqa: E402


def region(run, name, a, n, width=1):
    return run["r"][name][width * a: width * (a + n)]


def check_slices(run, sc, seed, ppm2, mix, slices):
    for s in slices:
        info = run["info"][s]
        m, n = info["m"], info["n"]
        a = info["off_col"]
        cnt = region(run, "COLCNT", a, n)
        gmin, gmax = region(run, "COLMIN", a, n), region(run, "COLMAX", a, n)
        g32 = np.where(cnt > 0, (gmax - gmin).astype(np.float32), np.float32(0))
        w = region(run, "WEIGHTS", a, n).astype(np.uint64)
        want = weights_from_g(g32.astype(np.float64), mix)
        assert np.array_equal(w, want), f"mix {mix} slice {s}: {int((w != want).sum())} weights differ"
        if mix > 0:
            assert (w >= 1).all()
        k1 = region(run, "OMEGA1", info["off1"], info["N1"])
        i1, j1 = keys_to_ij(k1)
        taken = np.zeros(m * n, bool)
        taken[i1 * n + j1] = True
        i2, j2, short = pass2(seed, s, m, n, info["N1"], ppm2, w, taken)
        n2 = int(run["stats"]["n2"][s])
        gi2, gj2 = keys_to_ij(region(run, "OMEGA2", info["off2"], n2))
        assert np.array_equal(gi2, i2) and np.array_equal(gj2, j2), f"mix {mix} slice {s}"
        assert bool(run["stats"]["flags"][s] & 4) == short


@pytest.mark.parametrize("mix", [0.3, 3.0, np.inf])
def test_tiny_mixed_weights_and_pass2(mix):
    sc = make_scene("tiny", 1)
    p = api.default_params(seed=1, pass1_ppm=50000, pass2_ppm=50000, max_iter=20, pass2_mix=mix)
    run = run_frame(sc, p, label=f"tiny mix {mix}")
    assert np.isfinite(run["radiance"]).all()
    check_slices(run, sc, 1, 50000, mix, range(sc.n_slices))


def test_mid_mixed_weights_and_pass2():
    sc = make_scene("mid", 11)
    p = api.default_params(seed=11, pass1_ppm=25000, pass2_ppm=25000, max_iter=5, pass2_mix=3.0)
    run = run_frame(sc, p, label="mid mix 3")
    rng = np.random.default_rng(3)
    slices = sorted(rng.choice(sc.n_slices, 6, replace=False).tolist())
    log(f"mid mix 3: slices {slices}")
    check_slices(run, sc, 11, 25000, 3.0, slices)


def test_mix_zero_is_the_papers_density():
    """pass2_mix = 0 renders bit-identically to the default parameters."""
    sc = make_scene("tiny", 1)
    base = dict(seed=1, pass1_ppm=50000, pass2_ppm=50000, max_iter=20)
    r0 = run_frame(sc, api.default_params(**base), regions=False, label="tiny default")
    r1 = run_frame(sc, api.default_params(pass2_mix=0.0, **base), regions=False, label="tiny mix 0")
    assert np.array_equal(r0["radiance"], r1["radiance"])
