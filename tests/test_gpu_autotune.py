"""Launch shapes of the batched step and the autotuner that picks one.

Every shape (1, 2 or 4 tiles per workgroup; one workgroup per tile group or a
persistent grid striding over them) must give bit-identical populations and
correlator sums, so the tuner's choice can never change a result; tuning
itself must leave the state untouched."""
import numpy as np
import pytest

from paper_1204_6734_amd import inputs as I

pytestmark = pytest.mark.gpu

SHAPES = [(1, 0), (2, 0), (4, 0), (1, 8), (2, 16), (4, 8), (1, 64), (2, 256)]


def ragged_members(F, prec, n=5, nx=70, ny=22, **extra):
    # 2 x 6 tiles per replica (the last tile column and row partly empty),
    # 60 tiles in all: not a multiple of 8 or of 4 tiles per workgroup
    out = []
    for m in I.ensemble_members(n, seed=3):
        out.append(F.make_params(nx, ny, precision=prec, ux0=m["ux0"], kT=m["kT"],
                                 seed=m["seed"], tau=I.mixed_taus(2), **extra))
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_every_launch_shape_is_bit_identical(flb, prec):
    precision = flb.FP32_SHIFTED if prec == "fp32" else flb.FP64
    ps = ragged_members(flb, precision, sample_every=3, block_steps=8)
    ref = flb.Ensemble(ps)
    ref.step(41)
    want = [(ref.populations(i), ref.covariance(i)) for i in range(len(ps))]
    for tpb, grid in SHAPES:
        print(f"shape tiles_per_block={tpb} grid_blocks={grid}", flush=True)
        E = flb.Ensemble(ps)
        E.set_launch(tpb, grid)
        assert E.get_launch() == {"tiles_per_block": tpb, "grid_blocks": grid}
        E.step(41)
        for i, (f, c) in enumerate(want):
            np.testing.assert_array_equal(E.populations(i), f)
            got = E.covariance(i)
            np.testing.assert_array_equal(got["cov_f"], c["cov_f"])
            np.testing.assert_array_equal(got["se_cov_f"], c["se_cov_f"])
            np.testing.assert_array_equal(got["mean_df"], c["mean_df"])
        E.close()


def test_launch_shape_with_structure_factor_and_graph(flb):
    """A lattice with S(k) sampling under a persistent shape, and an ensemble
    replayed from a graph under another, equal the default shape."""
    kw = dict(precision=flb.FP32_SHIFTED, ux0=0.1, kT=1e-4, seed=8, sample_every=2, sk_every=5)
    a = flb.Lattice(flb.make_params(96, 40, **kw))
    b = flb.Lattice(flb.make_params(96, 40, **kw))
    b.set_launch(4, 8)
    a.step(37)
    b.step(37)
    np.testing.assert_array_equal(a.populations(), b.populations())
    for w in (flb.SK_RHO, flb.SK_JX, flb.SK_JY):
        np.testing.assert_array_equal(a.structure_factor(w), b.structure_factor(w))
    ps = ragged_members(flb, flb.FP32_SHIFTED, sample_every=4, block_steps=12)
    e0 = flb.Ensemble(ps)
    e1 = flb.Ensemble(ps, graph_chunk=8)
    e1.set_launch(2, 16)
    for _ in range(3):
        e0.step(24)
        e1.step(24)
        e1.sync()
    for i in range(len(ps)):
        np.testing.assert_array_equal(e0.populations(i), e1.populations(i))
        np.testing.assert_array_equal(e0.covariance(i)["cov_f"], e1.covariance(i)["cov_f"])


def test_autotune_leaves_state_untouched(flb):
    ps = ragged_members(flb, flb.FP32_SHIFTED, n=8, nx=128, ny=64, sample_every=1,
                        block_steps=10)
    E = flb.Ensemble(ps)
    twin = flb.Ensemble(ps)
    E.step(15)
    twin.step(15)
    before = [E.populations(i) for i in range(len(ps))]
    cov_before = E.covariance(3)
    res = E.autotune(reps=2)
    print("autotune:", res)
    assert len(res) >= 3
    ms = [r["ms_per_step"] for r in res]
    assert ms == sorted(ms) and ms[0] > 0
    assert E.get_launch() == {k: res[0][k] for k in ("tiles_per_block", "grid_blocks")}
    assert E.t == 15
    for i in range(len(ps)):
        np.testing.assert_array_equal(E.populations(i), before[i])
    np.testing.assert_array_equal(E.covariance(3)["cov_f"], cov_before["cov_f"])
    # and the tuned run continues exactly like the untuned one
    E.step(20)
    twin.step(20)
    for i in range(len(ps)):
        np.testing.assert_array_equal(E.populations(i), twin.populations(i))
        np.testing.assert_array_equal(E.covariance(i)["cov_f"], twin.covariance(i)["cov_f"])
    # a new ensemble of the same kind starts with the tuned shape
    E2 = flb.Ensemble(ps)
    assert E2.get_launch() == E.get_launch()


def test_set_launch_rejects_bad_shapes(flb):
    L = flb.Lattice(flb.make_params(32, 32, kT=1e-4))
    for tpb, grid in [(3, 0), (0, 0), (8, 0), (1, -8), (1, 12)]:
        with pytest.raises(flb.FlbError) as e:
            L.set_launch(tpb, grid)
        assert e.value.code == flb.E_ARG


@pytest.mark.parametrize("nx,ny", [(1024, 1024), (100, 30)])
def test_copy_probe_measures_the_step_pattern(flb, nx, ny):
    """The no-arithmetic pass moves the step's bytes in a time of the right
    order, and leaves nothing behind (its own buffer)."""
    for prec, es in ((flb.FP32_SHIFTED, 4), (flb.FP64, 8)):
        ms = flb.copy_probe(nx, ny, prec, reps=5)
        gbps = 18 * es * nx * ny / (ms * 1e-3) / 1e9
        print(f"{nx}x{ny} step pattern, {es}-byte values: {ms:.4f} ms, {gbps:.0f} GB/s")
        assert 0 < ms < 100 and gbps > 10


def test_stream_copy_probe_measures_a_copy(flb):
    n = 256 << 20
    ms = flb.stream_copy_probe(n, reps=5)
    gbps = 2 * n / (ms * 1e-3) / 1e9
    print(f"contiguous copy of {n >> 20} MiB: {ms:.4f} ms, {gbps:.0f} GB/s")
    assert 0 < ms < 100 and gbps > 100
