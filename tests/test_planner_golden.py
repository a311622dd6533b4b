"""The planner's accounting against the paper's printed numbers.

* Equation 7 (tests/golden/eq7_coefficients.txt): `planner.predict` evaluates
  the printed polynomial with the coefficients in the printed order.
* Table 1 (tests/golden/table1_sample_sizes.txt): the total-time model the
  planner decides with -- preparation time, then the plain per-sample time
  divided by the prepared method's speedup -- explains the paper's measured
  speedups at four sample sizes: fitted on the 10 and 400 million columns, it
  predicts the 100 million column within 10 % and the 1 million column (the
  shortest, least certain runs) within a factor of 1.6, and its choice between
  the plain simulation and the prepared one agrees with the paper's measured
  speedup (above or below 1) at every network and sample size.
"""
import os

import numpy as np
import pytest

from paper_1605_00854_amd import planner

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(line.split())
    return out


def test_eq7_polynomial_with_the_printed_coefficients():
    b = [float(v) for _, v in _rows("eq7_coefficients.txt")]
    assert len(b) == 5
    for x1, x2 in [(0.0, 0.0), (0.5, 1.0), (0.9, 1.7), (0.3, 6.9), (0.68, 4.0)]:
        want = b[0] + b[1] * x1 + b[2] * x1 ** 2 + b[3] * x2 + b[4] * x2 ** 2
        assert planner.predict(x1, x2, b) == pytest.approx(want, rel=1e-12)


def _fit_row(prep, sp10, sp400):
    # speedup(N) = N t / (prep + N t / S)  <=>  1/speedup = (prep / N) (1/t) + 1/S
    A = np.array([[prep / 10.0, 1.0], [prep / 400.0, 1.0]])
    inv_t, inv_s = np.linalg.solve(A, np.array([1.0 / sp10, 1.0 / sp400]))
    return 1.0 / inv_t, 1.0 / inv_s


@pytest.mark.parametrize("row", _rows("table1_sample_sizes.txt"), ids=lambda r: f"net{r[0]}")
def test_total_time_model_explains_table_1(row):
    prep = float(row[4])
    sp = dict(zip((1, 10, 100, 400), (float(v) for v in row[5:9])))
    t_old, s = _fit_row(prep, sp[10], sp[400])          # seconds per million samples, asymptotic speedup
    assert t_old > 0 and s > 0
    for n_million in (1, 10, 100, 400):
        t = planner.predicted_times(work=float(n_million), plain_rate=1.0 / t_old, x1=0.0, x2=0.0,
                                    prep_reduction=prep, n_candidates=1, probe_work=0.0,
                                    coeffs=(s, 0.0, 0.0, 0.0, 0.0))
        predicted = t["plain"] / t["tuned"]
        if n_million == 100:
            assert predicted == pytest.approx(sp[n_million], rel=0.10)
        if n_million == 1:
            assert 1 / 1.6 < predicted / sp[n_million] < 1.6
        # the planner's choice between the plain and the prepared method
        assert (t["tuned"] < t["plain"]) == (sp[n_million] > 1.0)
