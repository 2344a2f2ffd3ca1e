"""Host logic of the autotuner: candidate sets and the amortisation of
rebuilds over their interval (no GPU)."""
import pytest

from paper_1606_02738_amd import autotune as AT


def _per(builds, t_build, refresh_ms=0.2):
    out, nb = [], 0
    for k in range(len(builds)):
        nb += builds[k]
        out.append({"n_builds": nb, "t_build_ms": t_build if builds[k] else refresh_ms})
    return out


def test_rebuild_every_step_is_plain_mean():
    per = _per([1] * 8, 10.0)
    assert AT.amortised_ms(240.0, per, 0, 10.0, 0) == pytest.approx(30.0)


def test_no_build_in_window_uses_half_the_skin():
    # 8 steps of 20 ms with no build; a cold build of 12 ms amortised over
    # rebuild_steps / 2 = 16 steps
    per = _per([0] * 8, 12.0)
    ms = AT.amortised_ms(160.0, per, 0, 12.0, 32)
    assert ms == pytest.approx(20.0 + 12.0 / 16.0)


def test_observed_interval_between_builds():
    # builds at steps 1 and 5 (interval 4), 10 ms each, the other steps 20 ms
    builds = [0, 1, 0, 0, 0, 1, 0, 0]
    per = _per(builds, 10.0)
    wall = 8 * 20.0 + 2 * 10.0
    ms = AT.amortised_ms(wall, per, 0, 99.0, 16)
    assert ms == pytest.approx(20.0 + 10.0 / 4.0)


def test_single_build_in_window():
    builds = [0, 0, 1, 0, 0, 0, 0, 0]
    per = _per(builds, 8.0)
    wall = 8 * 20.0 + 8.0
    ms = AT.amortised_ms(wall, per, 0, 99.0, 8)
    assert ms == pytest.approx(20.0 + 8.0 / 4.0)


def test_candidates_are_valid_combinations():
    for full in (False, True):
        cands = AT.candidates(full)
        assert cands
        for c in cands:
            # the gather force needs box pruning (symmetric lists)
            assert not (c["force"] == "gather" and c["prune"] != "box")
            assert c["exec_mode"] in ("grid", "persistent")
            assert (c["persistent_wgs"] > 0) == (c["exec_mode"] == "persistent")
            assert 1 <= c["n_split"] <= 64
    keys = {tuple(sorted(c.items())) for c in AT.candidates()}
    assert len(keys) == len(AT.candidates())


def test_kernel_candidates_sweep_each_axis_around_the_best():
    best = dict(n_split=64, exec_mode="persistent", persistent_wgs=2048, prune="box", use_graph=False,
                rebuild_steps=64, force="gather")
    cands = AT.kernel_candidates(best)
    assert len(cands) == 2 * len(AT.KERNEL_WAVES) + len(AT.KERNEL_BATCH)
    for c in cands:
        assert {k: c[k] for k in best} == best
        assert sum(1 for ax in ("waves_density", "waves_force", "batch") if c[ax]) == 1
    assert {c["waves_density"] for c in cands} == {0, *AT.KERNEL_WAVES}
    assert {c["batch"] for c in cands} == {0, *AT.KERNEL_BATCH}
