"""Host-side checks of the Python binding (no GPU needed).

The library takes raw device pointers with no buffer lengths, so the binding
refuses, before any library call, a train whose cores do not lie inside its
buffer, and any buffer that is not GPU memory.
"""
import numpy as np
import pytest
import torch

import paper_2410_19747_amd as T


def test_packed_tt_cores_must_lie_inside_the_buffer():
    data = torch.zeros(2 * 3 * 4, dtype=torch.float64)
    with pytest.raises(ValueError, match="needs 3 bonds"):
        T.PackedTT(data, [2, 3], [1, 2, 4, 1], [0, 4])
    with pytest.raises(ValueError, match="core 1"):
        T.PackedTT(data, [2, 3], [1, 2, 1], [0, 4 + 24])      # past the end
    with pytest.raises(ValueError, match="core 0"):
        T.PackedTT(data, [2, 3], [1, 2, 1], [-1, 4])          # negative offset
    with pytest.raises(ValueError, match="core 0"):
        T.PackedTT(data, [0, 3], [1, 2, 1], [0, 4])           # empty dimension


def test_packed_tt_refuses_host_memory():
    data = torch.zeros(2 + 6, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU tensor"):
        T.PackedTT(data, [2, 3], [1, 1, 1], [0, 2])
    with pytest.raises(ValueError, match="GPU tensor"):
        T.pack([np.ones((1, 2, 1)), np.ones((1, 3, 1))], device=torch.device("cpu"))


def test_workspace_refuses_host_memory():
    with pytest.raises(ValueError, match="GPU memory"):
        T.Workspace(torch.device("cpu")).get(1024)


def test_inner_loss_refuses_randomized_svd():
    """The loss's backward is the reverse mode of the full SVD's truncation,
    so a randomized swap SVD is refused before the forward product runs."""
    for mode in ("randomized", 1):
        with pytest.raises(T.TTMError, match="svd_mode") as e:
            T.ttm_inner_loss(None, None, None, 8, 1e-14, svd_mode=mode)
        assert e.value.code == T.TTM_EUNSUPPORTED
