"""The tolerance used where two FP32 accumulations of the same terms are compared
(float atomics): reordering passes, a missing or doubled term does not."""
import numpy as np
import pytest

from parity import assert_same_sums


def _terms():
    rng = np.random.default_rng(7)
    n_vert, n_terms = 500, 40000
    target = rng.integers(0, n_vert, n_terms)
    terms = (rng.standard_normal(n_terms) * 0.05).astype(np.float32)
    scale = np.zeros(n_vert)
    np.add.at(scale, target, np.abs(terms.astype(np.float64)))
    return n_vert, n_terms, target, terms, scale


def _sums(order_seed, drop=None, double=None):
    n_vert, n_terms, target, terms, _ = _terms()
    out = np.zeros(n_vert, dtype=np.float32)
    order = np.random.default_rng(order_seed).permutation(n_terms)
    for t in order:
        if t == drop:
            continue
        out[target[t]] += terms[t]
        if t == double:
            out[target[t]] += terms[t]
    return out


def test_reordered_sums_pass():
    assert_same_sums(_sums(1), _sums(2), _terms()[4])


@pytest.mark.parametrize("kind", ["drop", "double"])
def test_changed_term_fails(kind):
    a = _sums(1)
    b = _sums(2, drop=123) if kind == "drop" else _sums(2, double=123)
    with pytest.raises(AssertionError):
        assert_same_sums(a, b, _terms()[4])
