"""Host logic of the learned-guess driver (CPU tensors, no GPU): harvested
records are put in a canonical order that does not depend on the order in
which the sweep's waves appended them."""
import numpy as np
import torch

from paper_1607_02214_amd import learned


def test_canonical_order_is_lexicographic_and_independent_of_input_order():
    g = torch.Generator().manual_seed(0)
    R = torch.randint(0, 4, (5000, 28), generator=g).float()
    R[::7] = R[3]                                   # repeated records
    a = learned.canonical_order(R)
    b = learned.canonical_order(R[torch.randperm(R.shape[0], generator=g)])
    assert torch.equal(a, b)
    Rn = R.numpy()
    assert np.array_equal(a.numpy(), Rn[np.lexsort(Rn.T[::-1])])


def test_canonical_order_of_an_empty_buffer():
    R = torch.empty((0, 28))
    assert learned.canonical_order(R).shape == (0, 28)
