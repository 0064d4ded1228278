"""Host-side control flow of the subspace iteration (no GPU): the degree
back-off after a reported rank-deficient filtered block."""
import pytest


def _api():
    pytest.importorskip("torch")
    import paper_2110_15853_amd as P
    from paper_2110_15853_amd import _lib
    return P, _lib


def test_backoff_halves_until_the_pass_succeeds():
    P, L = _api()
    code = {v: k for k, v in L.STATUS.items()}["TTDFT_ERR_NOT_POSDEF"]
    tried, noted = [], []

    def run(deg):
        tried.append(deg)
        if deg > 50:
            raise L.TtdftError(code, "Cholesky breakdown")
        return "ok"

    deg, out = P.api.with_degree_backoff(run, 400, noted.append)
    assert (deg, out) == (50, "ok")
    assert tried == [400, 200, 100, 50] and noted == [400, 200, 100]


def test_backoff_gives_up_at_degree_one_and_passes_other_errors():
    P, L = _api()
    codes = {v: k for k, v in L.STATUS.items()}

    def always(deg):
        raise L.TtdftError(codes["TTDFT_ERR_NOT_POSDEF"], "Cholesky breakdown")

    with pytest.raises(L.TtdftError):
        P.api.with_degree_backoff(always, 5)

    def other(deg):
        raise L.TtdftError(codes["TTDFT_ERR_NONFINITE"], "nan")

    seen = []
    with pytest.raises(L.TtdftError):
        P.api.with_degree_backoff(other, 64, seen.append)
    assert seen == []                    # no retry for other errors
