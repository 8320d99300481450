"""Host-side logic of the Python binding (no device work): which storage of
a symmetric A is handed to the library in place, and the wanted count."""
import os

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2104_14186_amd", "libqdwhp.so")


def test_symmetric_storage_in_place_or_copied():
    import paper_2104_14186_amd as q
    n = 7
    B = torch.randn(n, n, dtype=torch.float64)
    A = B + B.t()
    assert q._sym_storage(A) is A                       # row-major: read in place
    At = A.t()
    assert q._sym_storage(At) is At                     # column-major view: in place
    big = torch.zeros(n, n + 3, dtype=torch.float64)
    big[:, :n] = A
    S = big[:, :n]
    C = q._sym_storage(S)                               # strided: a copy whose buffer is
    assert C is not S and C.is_contiguous() and torch.equal(C, S.t())   # A column by column
    # the buffers handed over in place hold the same numbers as the copy's
    for X in (A, At):
        assert torch.equal(torch.as_strided(X, (n * n,), (1,)), C.view(-1))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_count_matches_the_rounding_rule():
    import math
    import paper_2104_14186_amd as q
    for n in (1, 2, 7, 512, 16384):
        for f in (1e-6, 0.01, 0.1, 0.2, 0.5, 1.0):
            want = min(n, max(1, int(math.floor(f * n + 0.5))))
            assert q._count(n, f) == want, (n, f)
