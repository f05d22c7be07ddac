"""Host logic of the rectangular-field entry points (no GPU): the App. B
Taylor-degree rule of the library against the oracle's reading."""
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def mlcc():
    torch = pytest.importorskip("torch")   # noqa: F841
    from paper_2506_02121_amd import mlcc as m
    return m


@pytest.mark.parametrize("args", [(0.4, 2.0, 3.0, 1.3, 1e-6), (0.6, 10.0, 10.0, 1.5, 1e-9),
                                  (0.2, 7.0, 1.0, 2.0, 1e-4), (0.5, 32.0, 32.0, 1.2, 1e-6),
                                  (0.3, 5.0, 12.0, 1.8, 1e-12)])
def test_taylor_degree_matches_oracle(mlcc, args):
    assert mlcc.rect_taylor_degree(*args) == oracle.rect_taylor_degree(*args)


def test_taylor_degree_rejects_bad_arguments(mlcc):
    for args in [(0.0, 2.0, 3.0, 1.3, 1e-6), (0.4, 2.0, 3.0, 1.0, 1e-6),
                 (0.4, 2.0, 3.0, 1.3, 0.0), (0.4, 2.0, 3.0, 1.001, 1e-300)]:
        with pytest.raises(mlcc.MlccError):
            mlcc.rect_taylor_degree(*args)


def test_rect_workload_uses_app_b_degree(mlcc):
    """The rect workload's Taylor degree is the App. B rule's for error 1e-8
    where |z| < |c| / 1.25."""
    from paper_2506_02121_amd import fields
    f = fields.workload("rect").field
    ks, c1, c2, t = f.sheet
    assert t == mlcc.rect_taylor_degree(ks, c1, c2, 1.25, 1e-8) == oracle.rect_taylor_degree(
        ks, c1, c2, 1.25, 1e-8)
    # the corner sits 1.25 times beyond the corner of the star-free image of the
    # 40 x 40 source map, |x| <= 20 / 1.3, |y| <= 20 / 0.7 (to the rounding of N)
    assert abs(np.hypot(c1, c2) / (1.25 * np.hypot(20 / 1.3, 20 / 0.7)) - 1) < 2e-3
    assert abs(c2 / c1 - 1.3 / 0.7) < 1e-12
