"""Host-side logic of the learned selector's training loop (no GPU): the
per-kind gather cost fit and the decision-threshold search."""
import numpy as np

from paper_1806_08092_amd import MLP_IN
from paper_1806_08092_amd.learned import Samples, calibrate_offset, relabel_by_id_kind


def _samples(rng, n_it=40, rows_per_it=5, c_sc=7e-5, c_pc=4e-6):
    sc_ids = rng.integers(0, 2_000_000, n_it).astype(np.float64)
    pc_ids = rng.integers(0, 20_000_000, n_it).astype(np.float64)
    g_us = c_sc * sc_ids + c_pc * pc_ids
    n = n_it * rows_per_it
    x = np.zeros((n, MLP_IN), np.float32)
    ea = rng.integers(0, 50_000, n).astype(np.float64)
    ep = rng.integers(0, 400_000, n).astype(np.float64)
    x[:, 1] = np.log1p(ea)
    x[:, 2] = np.log1p(ep)
    s_sc = rng.random(n).astype(np.float32) * 10
    s_pc = rng.random(n).astype(np.float32) * 10
    it = np.repeat(np.arange(n_it, dtype=np.int32), rows_per_it)
    return Samples(x, s_sc.copy(), s_pc.copy(), it, [], [], s_sc, s_pc, g_us, sc_ids, pc_ids), ea, ep


def test_relabel_recovers_per_kind_costs():
    rng = np.random.default_rng(5)
    data, ea, ep = _samples(rng)
    out, c_sc, c_pc = relabel_by_id_kind(data)
    assert abs(c_sc - 7e-5) < 1e-9 and abs(c_pc - 4e-6) < 1e-10
    np.testing.assert_allclose(out.t_sc, data.s_sc + 7e-5 * ea, rtol=1e-4, atol=1e-4)
    np.testing.assert_allclose(out.t_pc, data.s_pc + 4e-6 * ep, rtol=1e-4, atol=1e-4)
    # the scatter-only times and per-iteration records are carried over
    assert out.s_sc is data.s_sc and out.g_us is data.g_us


def test_relabel_costs_never_negative():
    # gather time that falls as source-centric ids rise: the fit clamps that
    # kind's cost at zero instead of rewarding source-centric mode
    rng = np.random.default_rng(6)
    data, _, ep = _samples(rng, c_sc=0.0)
    data.g_us = 4e-6 * data.g_pc_ids - 1e-7 * data.g_sc_ids
    out, c_sc, c_pc = relabel_by_id_kind(data)
    assert c_sc == 0.0 and c_pc > 0.0
    np.testing.assert_allclose(out.t_sc, data.s_sc, rtol=0, atol=0)


def test_concat_offsets_iteration_index():
    rng = np.random.default_rng(7)
    a, _, _ = _samples(rng, n_it=3, rows_per_it=2)
    b, _, _ = _samples(rng, n_it=4, rows_per_it=2)
    c = Samples.concat([a, b])
    assert len(c) == len(a) + len(b)
    assert list(c.it) == list(a.it) + list(b.it + 3)
    assert np.array_equal(c.g_us[c.it[len(a):]], b.g_us[b.it])


class _FakeMlp:
    """Records the output-bias offset the search leaves in the model."""
    def __init__(self):
        self.offset = 0.0

    def shift_logit(self, delta, stream=None):
        self.offset += delta


def _search(times, min_gain=0.01):
    m = _FakeMlp()
    offs = tuple(times)
    best, res = calibrate_offset(m, lambda: times[m.offset], offsets=offs, min_gain=min_gain)
    assert m.offset == best
    assert set(res) == set(offs) | {0.0}
    return best


def test_calibrate_offset_keeps_zero_within_noise():
    # 16 is fastest by 0.1%: less than the 1% it must win by
    assert _search({-2.0: 53.0, 0.0: 53.02, 1.0: 53.1, 16.0: 52.97}) == 0.0


def test_calibrate_offset_moves_on_a_real_gain():
    assert _search({-2.0: 53.0, 0.0: 53.0, 4.0: 50.0, 8.0: 51.0}) == 4.0
    # ties go to the offset nearer zero
    assert _search({-1.0: 50.0, 0.0: 53.0, 1.0: 50.0, 2.0: 50.0}) in (-1.0, 1.0)


def test_calibrate_offset_times_zero_when_not_listed():
    m = _FakeMlp()
    seen = []

    def run():
        seen.append(m.offset)
        return {1.0: 60.0, 2.0: 40.0, 0.0: 50.0}[m.offset]

    best, res = calibrate_offset(m, run, offsets=(1.0, 2.0))
    assert seen == [1.0, 2.0, 0.0]
    assert best == 2.0 and m.offset == 2.0 and res[0.0] == 50.0
