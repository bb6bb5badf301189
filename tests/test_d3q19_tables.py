"""The D3Q19 step's constant tables (csrc/d3q19_tables.hpp) against their
generator and the properties the kernel relies on: the committed header is
what gen_d3q19.py writes; the basis rows are orthonormal under the weights,
each row exactly even or odd in the velocity (the kernel folds sums over a
velocity and its opposite, and checks this at compile time); and the
polynomial tables give the Gram entries <m^a, m^b>_g and pi_b = <1, m^b>_g
at random velocities."""
import importlib.util
import os

import numpy as np

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_1204_6734_amd", "csrc")


def generator():
    spec = importlib.util.spec_from_file_location("gen_d3q19", os.path.join(CSRC, "gen_d3q19.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_committed_header_is_the_generators_output(tmp_path):
    g = generator()
    out = tmp_path / "d3q19_tables.hpp"
    g.write(str(out))
    with open(os.path.join(CSRC, "d3q19_tables.hpp")) as fh:
        assert fh.read() == out.read_text()


def test_rows_orthonormal_and_of_definite_parity():
    g = generator()
    m = g.basis()
    gram = np.einsum("i,ai,bi->ab", g.W, m, m)
    assert np.abs(gram - np.eye(19)).max() < 1e-14
    opp = [int(np.where((g.C == -g.C[i]).all(1))[0][0]) for i in range(19)]
    assert opp == [0] + [k + 1 if k % 2 else k - 1 for k in range(1, 19)]
    for b in range(19):
        even = np.array_equal(m[b][opp], m[b])
        odd = np.array_equal(m[b][opp], -m[b])
        assert even or odd, b
        if odd:
            assert m[b][0] == 0.0


def test_polynomial_tables_give_the_gram_entries():
    g = generator()
    m, G, Pi = g.tables()
    rng = np.random.default_rng(4)
    for _ in range(5):
        u = rng.uniform(-0.2, 0.2, 3)
        cu = g.C @ u
        gw = g.W * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u @ u)
        mono = np.array([u[0], u[1], u[2], u[0] ** 2, u[1] ** 2, u[2] ** 2,
                         u[0] * u[1], u[0] * u[2], u[1] * u[2]])
        want = np.einsum("i,ai,bi->ab", gw, m, m)
        got = np.eye(19) * (1 - 1.5 * u @ u) + G @ mono
        assert np.abs(got - want).max() < 1e-13
        assert np.abs(Pi @ mono - (m @ gw - np.eye(19)[0]))[1:].max() < 1e-13
