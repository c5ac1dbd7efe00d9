"""Host-side checks of the Python binding (no GPU): caller-supplied outputs
and fields are validated before any launch, and a non-OK solve status is
raised, not returned."""
import pytest
import torch

import paper_2410_14917_amd as kp
from paper_2410_14917_amd import _check_vec


def test_check_vec_rejects_wrong_outputs_before_any_launch():
    ok = torch.zeros(12, dtype=torch.float64)
    with pytest.raises(ValueError, match="float64"):
        _check_vec("out", ok.float(), 12)
    with pytest.raises(ValueError, match="contiguous"):
        _check_vec("out", torch.zeros(24, dtype=torch.float64)[::2], 12)
    with pytest.raises(ValueError, match="12 elements"):
        _check_vec("out", torch.zeros(11, dtype=torch.float64), 12)
    with pytest.raises(ValueError, match="device tensor"):
        _check_vec("out", ok, 12)                 # a host tensor
    with pytest.raises(ValueError, match="torch tensor"):
        _check_vec("out", [0.0] * 12, 12)


def test_operator_fields_are_checked():
    op = kp.Operator(kp.KP_OP_ALLEN_CAHN, 4, 3, nu=0.01,
                     field0=torch.zeros(11, dtype=torch.float64))
    with pytest.raises(ValueError, match="12 elements"):
        op.c_struct()
    op.field0 = torch.zeros(12, dtype=torch.float32)
    with pytest.raises(ValueError, match="float64"):
        op.c_struct()


def test_status_is_raised():
    assert kp.raise_on_status({"status": 0})["status"] == 0
    for st in (1, 2, 3):
        with pytest.raises(kp.SolveError) as e:
            kp.raise_on_status({"status": st, "substeps": 7})
        assert e.value.info["status"] == st


def test_single_row_B_gets_a_valid_leading_dimension():
    """A (1, N) view whose row stride is 1 (a transposed numpy column): the
    leading dimension passed to the library is N."""
    import numpy as np
    from paper_2410_14917_amd import _b_layout
    col = np.zeros((12, 1))
    B = torch.as_tensor(np.ascontiguousarray(col.T))
    assert _b_layout(B, 12) == (0, 12)
    assert _b_layout(torch.zeros((3, 12), dtype=torch.float64), 12) == (2, 12)
    assert _b_layout(torch.zeros((3, 16), dtype=torch.float64)[:, :12], 12) == (2, 16)
    with pytest.raises(ValueError):
        _b_layout(torch.zeros((12, 3), dtype=torch.float64).T, 12)   # not unit stride
    with pytest.raises(ValueError):
        _b_layout(torch.zeros((3, 11), dtype=torch.float64), 12)
