"""Host logic of the EM driver objects (no GPU): the annealing schedules and
the argument checks of the model objects."""
import pytest

from paper_1908_06843_amd.em import BSC_ET, LinearAnnealing


def test_linear_annealing_schedule():
    a = LinearAnnealing(5, beta_start=0.2, noise_start=0.1, anneal_steps=3)
    assert [round(a.beta(i), 12) for i in range(5)] == [0.2, 0.6, 1.0, 1.0, 1.0]
    assert [round(a.noise(i), 12) for i in range(5)] == [0.1, 0.05, 0.0, 0.0, 0.0]
    b = LinearAnnealing(4)
    assert all(b.beta(i) == 1.0 and b.noise(i) == 0.0 for i in range(4))
    assert LinearAnnealing(1, beta_start=0.5).beta(0) == 1.0


@pytest.mark.parametrize("kw", [dict(iterations=0), dict(iterations=3, beta_start=0.0),
                                dict(iterations=3, beta_start=1.5),
                                dict(iterations=3, noise_start=-1.0)])
def test_linear_annealing_rejects(kw):
    with pytest.raises(ValueError):
        LinearAnnealing(**kw)


@pytest.mark.parametrize("Hp,gamma", [(0, 0), (11, 2), (4, 5), (33, 2)])
def test_model_rejects_truncation(Hp, gamma):
    with pytest.raises(ValueError):
        BSC_ET(25, 10 if Hp != 33 else 40, Hp, gamma, device=0)


def test_dsc_model_checks_its_value_set():
    from paper_1908_06843_amd import em
    m = em.DSC_ET(16, 8, 4, 2, (0.0, 1.0, -1.0), device=0)
    assert m.kind == "dsc" and m._nvalues() == 3
    assert m._theta({"pv": (0.8, 0.1, 0.1), "sigma": 0.5}) == pytest.approx(
        [0.2, 0.5, 0.8, 0.1, 0.1])
    with pytest.raises(ValueError):
        em.DSC_ET(16, 8, 4, 2, (1.0, 2.0), device=0)
    with pytest.raises(ValueError):
        em.DSC_ET(16, 8, 4, 2, (0.0,), device=0)


def test_selected_points_needs_a_linear_model():
    from paper_1908_06843_amd import em
    with pytest.raises(ValueError):
        em.EM(em.MCA_ET(16, 8, 4, 2, device=0), LinearAnnealing(2), selected_points=True)
