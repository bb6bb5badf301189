"""GPU tests of the batched execution patterns: ensembles in one launch
(eager and hipGraph replay) and the continuous-batching server.  Each
replica or request must give the same result as running it alone."""
import numpy as np
import pytest

from paper_1204_6734_amd import inputs as I

pytestmark = pytest.mark.gpu


def members(F, n, nx, ny, prec, **extra):
    out = []
    for m in I.ensemble_members(n, seed=3):
        out.append(F.make_params(nx, ny, precision=prec, ux0=m["ux0"], kT=m["kT"],
                                 seed=m["seed"], **extra))
    return out


@pytest.mark.parametrize("chunk", [0, 8])
def test_ensemble_replicas_equal_alone(flb, chunk):
    ps = members(flb, 5, 70, 20, flb.FP32_SHIFTED, sample_every=1, block_steps=16)
    E = flb.Ensemble(ps, graph_chunk=chunk)
    E.step(53)
    for i in (0, 2, 4):
        L = flb.Lattice(ps[i])
        L.step(53)
        np.testing.assert_array_equal(E.populations(i), L.populations())
        ce, cl = E.covariance(i), L.covariance()
        assert ce["nblocks"] == cl["nblocks"] == 3
        np.testing.assert_array_equal(ce["cov_f"], cl["cov_f"])
        np.testing.assert_array_equal(ce["se_cov_f"], cl["se_cov_f"])


def test_ensemble_block_closes_in_and_out_of_step_equal_alone(flb):
    """Replicas that close their time blocks together are closed by one
    batched launch; replicas whose blocks or sampling differ, and closes that
    first merge full record lists, take one launch each.  Mixed ensembles
    (every replica closing each sample, with merges of the records; and
    block lengths 3, 3 and 5 with sampling every 1, 1 and 2) against the
    same lattices alone: correlator sums, standard errors and block counts
    bit for bit."""
    cases = [[dict(sample_every=1, block_steps=1)] * 3,
             [dict(sample_every=1, block_steps=3), dict(sample_every=1, block_steps=3),
              dict(sample_every=2, block_steps=5)]]
    for steps, extras in ((1100, cases[0]), (97, cases[1])):
        ps = [flb.make_params(16, 8, precision=flb.FP32_SHIFTED, ux0=0.05 * k, kT=1e-4,
                              seed=500 + k, **e) for k, e in enumerate(extras)]
        E = flb.Ensemble(ps, graph_chunk=0)
        E.step(steps)
        for i, p in enumerate(ps):
            L = flb.Lattice(p)
            L.step(steps)
            ce, cl = E.covariance(i), L.covariance()
            assert ce["nblocks"] == cl["nblocks"] and ce["nsamples"] == cl["nsamples"]
            for k in ("mean_df", "cov_f", "se_cov_f", "se_cov_m"):
                np.testing.assert_array_equal(ce[k], cl[k], err_msg=f"replica {i} {k}")
            L.close()
        E.close()


def test_ensemble_graph_replay_equals_eager(flb):
    ps = members(flb, 4, 128, 128, flb.FP32_SHIFTED, sample_every=1, block_steps=40)
    a = flb.Ensemble(ps, graph_chunk=20)
    b = flb.Ensemble(ps, graph_chunk=0)
    for _ in range(3):  # replays interleaved with eager work and syncs
        a.step(60)
        b.step(60)
        a.sync()
        b.sync()
        for i in range(4):
            np.testing.assert_array_equal(a.populations(i), b.populations(i))
            np.testing.assert_array_equal(a.covariance(i)["cov_f"], b.covariance(i)["cov_f"])


@pytest.mark.parametrize("prec,nx,ny", [("fp64", 96, 40), ("fp32", 96, 40), ("fp32", 32, 32)])
def test_lattice_graph_replay_equals_eager(flb, prec, nx, ny):
    """A lattice replaying captured graphs of 20 steps, with the correlator
    samples of every step and a structure-factor transform every 10 steps
    inside them, against the same lattice launched eagerly: populations,
    correlator sums, time blocks (closing every 30 samples, which replays
    may not straddle) and structure factors are bit-identical after every
    call of a schedule of odd lengths (eager steps up to the next multiple
    of 20, replays, eager remainders), with host synchronisations between
    the replays, and again after a statistics reset."""
    precision = flb.FP64 if prec == "fp64" else flb.FP32_SHIFTED
    kw = dict(precision=precision, ux0=0.1, kT=1e-4, tau=I.mixed_taus(2), seed=5,
              sample_every=1, sk_every=10, block_steps=30)
    a = flb.Lattice(flb.make_params(nx, ny, **kw))
    b = flb.Lattice(flb.make_params(nx, ny, **kw))
    b.set_graph_chunk(20)

    def same():
        a.sync()
        b.sync()
        np.testing.assert_array_equal(a.populations(), b.populations())
        ca, cb = a.covariance(), b.covariance()
        for k, v in ca.items():
            np.testing.assert_array_equal(v, cb[k], err_msg=k)
        for w in range(5):
            np.testing.assert_array_equal(a.structure_factor(w), b.structure_factor(w))

    for n in (7, 33, 40, 1, 59, 20, 20):
        a.step(n)
        b.step(n)
        same()
    a.reset_stats()
    b.reset_stats()
    for n in (3, 77):
        a.step(n)
        b.step(n)
        same()
    assert a.covariance()["nsamples"] == 80 * nx * ny
    a.close()
    b.close()


def _serve(F, reqs, budget, slots=8, chunk=50):
    S = F.Server(budget, max_slots=slots, chunk_steps=chunk, threaded=False)
    ids = {}
    for k, (p, n) in enumerate(reqs):
        ids[S.submit(p, n, tag=k)] = k
    S.drain()
    res = {r["tag"]: r for r in S.poll(len(reqs) + 4)}
    S.close()
    assert len(res) == len(reqs)
    return res


def test_server_result_alone_equals_in_mix(flb):
    reqs = []
    for k, (side, n, kT, ux) in enumerate([(64, 180, 1e-4, 0.1), (100, 75, 1e-3, 0.0),
                                          (37, 333, 1e-5, 0.2), (64, 50, 2e-4, 0.05),
                                          (90, 260, 5e-4, 0.15), (128, 120, 1e-4, 0.12)]):
        p = flb.make_params(side, side, ux0=ux, kT=kT, seed=100 + k, sample_every=1,
                            block_steps=20)
        reqs.append((p, n))
    # small budget and few slots: requests queue, join and leave mid-stream
    budget = 3 * flb.Server.request_bytes(reqs[-1][0])
    mix = _serve(flb, reqs, budget, slots=3, chunk=40)
    for k, (p, n) in enumerate(reqs):
        alone = _serve(flb, [(p, n)], budget, slots=1, chunk=40)[0]
        m = mix[k]
        assert m["status"] == 0 and alone["status"] == 0
        assert m["cov"]["nsamples"] == n * p.nx * p.ny
        np.testing.assert_array_equal(m["cov"]["cov_f"], alone["cov"]["cov_f"])
        np.testing.assert_array_equal(m["cov"]["mean_df"], alone["cov"]["mean_df"])


def test_server_matches_lattice(flb):
    p = flb.make_params(80, 48, ux0=0.1, kT=1e-4, seed=42, sample_every=1, block_steps=25)
    r = _serve(flb, [(p, 150)], 64 << 20)[0]
    L = flb.Lattice(p)
    L.step(150)
    c = L.covariance()
    np.testing.assert_array_equal(r["cov"]["cov_f"], c["cov_f"])


def test_threaded_server_completes_everything(flb):
    S = flb.Server(256 << 20, max_slots=4, chunk_steps=25, threaded=True)
    for k in range(10):
        p = flb.make_params(32 + 8 * k, 40, ux0=0.01 * k, kT=1e-4, seed=k, sample_every=1)
        S.submit(p, 30 + 10 * k, tag=k)
    S.drain()
    res = S.poll(32)
    assert sorted(r["tag"] for r in res) == list(range(10))
    assert all(r["status"] == 0 for r in res)
    assert all(r["t_submit"] <= r["t_admit"] <= r["t_done"] for r in res)
    st = S.stats()
    assert st["completed"] == 10 and st["queued"] == 0


def test_ensemble_replica_matches_oracle(flb):
    """An FP64 ensemble of ragged lattices (tile count not a multiple of the
    eight XCDs) against the oracle, replica by replica."""
    import oracle as O
    taus = I.mixed_taus(2)
    ps, os_ = [], []
    for k, ux in enumerate([0.0, 0.12, 0.2]):
        kw = dict(ux0=ux, kT=1e-4, tau=taus, seed=30 + k)
        ps.append(flb.make_params(37, 11, precision=flb.FP64, **kw))
        os_.append(O.Lattice(O.make_params(37, 11, **kw)))
    E = flb.Ensemble(ps, graph_chunk=4)
    E.step(23)
    for k, o in enumerate(os_):
        o.step(23)
        f = o.populations()
        assert np.abs(E.populations(k) - f).max() <= 1e-12 * np.abs(f).max()


def test_server_request_matches_oracle(flb):
    import oracle as O
    kw = dict(ux0=0.1, kT=1e-4, seed=77, sample_every=1, block_steps=10)
    p = flb.make_params(29, 13, precision=flb.FP64, **kw)
    S = flb.Server(64 << 20, max_slots=4, chunk_steps=6, precision=flb.FP64, threaded=False)
    S.submit(p, 40, tag=1)
    S.submit(flb.make_params(50, 50, precision=flb.FP64, kT=1e-4, seed=3, sample_every=1), 17)
    S.drain()
    r = [x for x in S.poll(8) if x["tag"] == 1][0]
    o = O.Lattice(O.make_params(29, 13, **kw))
    o.step(40)
    co = o.covariance()
    assert r["cov"]["nsamples"] == co["nsamples"]
    assert np.abs(r["cov"]["cov_f"] - co["cov_f"]).max() <= 1e-10 * np.abs(co["cov_f"]).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sampling_variant_does_not_change_the_trajectory(flb, prec):
    """The sampling kernel variant and the plain one update identically, so a
    request's populations do not depend on whether others sample."""
    precision = flb.FP64 if prec == "fp64" else flb.FP32_SHIFTED
    kw = dict(precision=precision, ux0=0.1, kT=1e-4, tau=I.mixed_taus(2), seed=12)
    a = flb.Lattice(flb.make_params(66, 18, sample_every=1, **kw))
    b = flb.Lattice(flb.make_params(66, 18, sample_every=0, **kw))
    a.step(31)
    b.step(31)
    np.testing.assert_array_equal(a.populations(), b.populations())


def test_ensemble_graph_with_sampling_interval(flb):
    """Replays with a sampling interval > 1 and time blocks that do not line up
    with the replay chunk equal the eager single-lattice runs."""
    ps = members(flb, 3, 64, 24, flb.FP32_SHIFTED, sample_every=5, block_steps=7)
    E = flb.Ensemble(ps, graph_chunk=10)
    E.step(3)      # misalign first
    E.step(120)
    for i in range(3):
        L = flb.Lattice(ps[i])
        L.step(123)
        np.testing.assert_array_equal(E.populations(i), L.populations())
        ce, cl = E.covariance(i), L.covariance()
        assert ce["nsamples"] == cl["nsamples"] == 25 * 64 * 24
        assert ce["nblocks"] == cl["nblocks"] == 3
        np.testing.assert_array_equal(ce["cov_f"], cl["cov_f"])


def test_server_mixed_compute_classes_alone_equals_in_mix(flb):
    """Requests above |u0| = 0.25 run in the FP64-compute class, the others in
    FP32; both classes advance together and each result equals its solo run
    and the single-lattice run of the same parameters."""
    reqs = []
    for k, (side, n, ux) in enumerate([(48, 90, 0.3), (64, 60, 0.1), (40, 120, 0.28),
                                       (56, 70, 0.0)]):
        p = flb.make_params(side, side, ux0=ux, kT=1e-4, seed=200 + k, sample_every=1,
                            block_steps=10)
        reqs.append((p, n))
    budget = 64 << 20
    mix = _serve(flb, reqs, budget, slots=4, chunk=20)
    for k, (p, n) in enumerate(reqs):
        alone = _serve(flb, [(p, n)], budget, slots=1, chunk=20)[0]
        np.testing.assert_array_equal(mix[k]["cov"]["cov_f"], alone["cov"]["cov_f"])
        L = flb.Lattice(p)
        L.step(n)
        np.testing.assert_array_equal(mix[k]["cov"]["cov_f"], L.covariance()["cov_f"])


@pytest.mark.parametrize("chunk", [0, 6])
def test_ensemble_mixed_compute_classes_equal_alone(flb, chunk):
    """Replicas above |u0| = 0.25 (FP64 collision on FP32 storage) and below
    it (FP32 collision) in one ensemble: two launches per step, and every
    replica equals its own single-lattice run."""
    ps = [flb.make_params(40, 12, ux0=ux, kT=1e-4, seed=300 + k, sample_every=2, block_steps=6)
          for k, ux in enumerate([0.1, 0.3, 0.0, 0.27, 0.2])]
    E = flb.Ensemble(ps, graph_chunk=chunk)
    E.step(25)
    for i, p in enumerate(ps):
        L = flb.Lattice(p)
        L.step(25)
        np.testing.assert_array_equal(E.populations(i), L.populations())
        np.testing.assert_array_equal(E.covariance(i)["cov_f"], L.covariance()["cov_f"])


def test_server_failing_request_leaves_the_others_unchanged(flb):
    """A request whose thermal start at a high temperature leaves the validity
    region reports FLB_E_INVALID_VELOCITY; the requests batched with it give
    the same results as when they run alone."""
    good = [(flb.make_params(48, 40, ux0=0.1, kT=1e-4, seed=400 + k, sample_every=1,
                             block_steps=10), 60) for k in range(2)]
    bad = (flb.make_params(40, 40, kT=0.05, seed=7, init=flb.INIT_THERMAL, sample_every=1), 60)
    reqs = [good[0], bad, good[1]]
    mix = _serve(flb, reqs, 64 << 20, slots=3, chunk=20)
    assert mix[1]["status"] == flb.E_INVALID_VELOCITY
    for k in (0, 2):
        alone = _serve(flb, [reqs[k]], 64 << 20, slots=1, chunk=20)[0]
        assert mix[k]["status"] == alone["status"] == 0
        np.testing.assert_array_equal(mix[k]["cov"]["cov_f"], alone["cov"]["cov_f"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_server_odd_step_count_equals_lattice(flb, prec):
    """A request of an odd number of steps (the server's chunks are even, so
    it stops inside a chunk) with time blocks that end inside chunks: its
    correlators equal the single lattice's bit for bit, in both storage
    precisions."""
    precision = flb.FP64 if prec == "fp64" else flb.FP32_SHIFTED
    kw = dict(precision=precision, ux0=0.1, kT=1e-4, tau=I.mixed_taus(2), seed=21,
              sample_every=1, block_steps=7)
    p = flb.make_params(29, 13, **kw)  # 1 x 4 tiles
    L = flb.Lattice(p)
    L.step(301)
    c = L.covariance()
    S = flb.Server(64 << 20, max_slots=2, chunk_steps=10, precision=precision, threaded=False)
    S.submit(p, 301, tag=1)
    S.drain()
    r = S.poll(4)[0]
    S.close()
    assert r["status"] == 0 and r["cov"]["nsamples"] == c["nsamples"] == 301 * 29 * 13
    np.testing.assert_array_equal(r["cov"]["cov_f"], c["cov_f"])
    np.testing.assert_array_equal(r["cov"]["mean_df"], c["mean_df"])
