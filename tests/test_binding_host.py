"""Host-side argument checks of the Python binding: bad batch arguments raise
ValueError before the library sees a pointer (no GPU needed)."""

import pytest
import torch

from paper_1807_04638_amd import lddmm as B


class _Ctx:
    def __init__(self, n, dtype=torch.float32):
        self.n, self.dtype, self.device = tuple(n), dtype, torch.device("cuda:0")


def _batch(sizes):
    b = object.__new__(B.Batch)  # no device work: only the per-pair metadata the checks read
    b.contexts = [_Ctx(n) for n in sizes]
    b.device = torch.device("cuda:0")
    b.lib = None
    return b


def test_batch_rejects_a_short_list():
    b = _batch([(8, 8, 8), (8, 8, 10)])
    with pytest.raises(ValueError, match="2 pairs"):
        b.gn_solve([torch.zeros(3, 8, 8, 8)])
    with pytest.raises(ValueError, match="2 pairs"):
        b.hessvec([torch.zeros(3, 8, 8, 8)] * 3, [torch.zeros(3, 8, 8, 8)] * 2)


@pytest.mark.parametrize(
    "bad, what",
    [
        (torch.zeros(3, 8, 8, 12), "shape"),
        (torch.zeros(3, 8, 8, 10, dtype=torch.float64), "dtype"),
        (torch.zeros(3, 8, 8, 10), "device"),  # a host tensor
        (None, "missing"),
    ],
)
def test_batch_rejects_bad_fields(bad, what):
    b = _batch([(8, 8, 8), (8, 8, 10)])
    good = torch.zeros(3, 8, 8, 8)
    with pytest.raises(ValueError):
        b._fields([good, bad], "v0s")
    with pytest.raises(ValueError):
        b.hessvec([good, bad], [good, bad])


def test_batch_rejects_non_contiguous_fields():
    b = _batch([(8, 8, 8)])
    t = torch.zeros(3, 8, 8, 8).transpose(2, 3)
    with pytest.raises(ValueError):
        b._fields([t], "dvs")
