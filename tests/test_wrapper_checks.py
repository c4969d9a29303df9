"""The Python wrappers reject tensors the kernels would misread before any
library call or launch: CPU tensors, mixed devices, b of another dtype or
length, strided b, x that is not contiguous float64 of length n, column-major
A, and malformed CSR arrays."""
import pytest

torch = pytest.importorskip("torch")

import paper_2409_14309_amd as sns  # noqa: E402


def _ok():
    A = torch.zeros(50, 4, dtype=torch.float32)
    b = torch.zeros(50, dtype=torch.float32)
    x = torch.zeros(4, dtype=torch.float64)
    return A, b, x


def test_valid_arguments_pass_the_shape_checks():
    A, b, x = _ok()
    assert sns.check_args(A, b, x, need_cuda=False) == (50, 4)
    # a row-padded view of a wider matrix is a valid dense A
    W = torch.zeros(50, 8, dtype=torch.float64)
    assert sns.check_args(W[:, :4], torch.zeros(50, dtype=torch.float64), need_cuda=False) == (50, 4)


def test_cpu_tensors_are_rejected_before_any_library_call():
    A, b, x = _ok()
    with pytest.raises(ValueError, match="GPU memory"):
        sns.check_args(A, b, x)
    with pytest.raises(ValueError, match="GPU memory"):
        sns.lstsq(A, b, "count", 8, 1)
    with pytest.raises(ValueError, match="GPU memory"):
        sns.sketch(A, b, "count", 8, 1)
    with pytest.raises(ValueError, match="GPU memory"):
        sns.lstsq_batched([A], [b], [8], [1])


@pytest.mark.parametrize("case", ["b_dtype", "b_len", "b_strided", "x_dtype", "x_len",
                                  "x_strided", "A_int", "A_colmajor", "A_1d"])
def test_bad_dense_arguments(case):
    A, b, x = _ok()
    if case == "b_dtype":
        b = b.double()
    elif case == "b_len":
        b = torch.zeros(49, dtype=torch.float32)
    elif case == "b_strided":
        b = torch.zeros(50, 2, dtype=torch.float32)[:, 0]
    elif case == "x_dtype":
        x = x.float()
    elif case == "x_len":
        x = torch.zeros(5, dtype=torch.float64)
    elif case == "x_strided":
        x = torch.zeros(4, 2, dtype=torch.float64)[:, 1]
    elif case == "A_int":
        A = torch.zeros(50, 4, dtype=torch.int32)
    elif case == "A_colmajor":
        A = torch.zeros(4, 50, dtype=torch.float32).t()
    elif case == "A_1d":
        A = torch.zeros(50, dtype=torch.float32)
    with pytest.raises(ValueError):
        sns.check_args(A, b, x, need_cuda=False)


def test_bad_csr_arguments():
    rp = torch.tensor([0, 1, 2], dtype=torch.int32)
    ci = torch.tensor([0, 1], dtype=torch.int32)
    v = torch.tensor([1.0, 2.0], dtype=torch.float32)
    ok = sns.CsrMatrix(rp, ci, v, (2, 3))
    assert sns.check_args(ok, torch.zeros(2), need_cuda=False) == (2, 3)
    bad = [sns.CsrMatrix(rp.long(), ci, v, (2, 3)),                 # int64 row_ptr
           sns.CsrMatrix(rp, ci, v, (3, 3)),                        # row_ptr too short
           sns.CsrMatrix(rp, ci[:1], v, (2, 3)),                    # col_idx / values mismatch
           sns.CsrMatrix(rp, ci, v.half(), (2, 3))]                 # values dtype
    for A in bad:
        with pytest.raises(ValueError):
            sns.check_args(A, None, need_cuda=False)
    with pytest.raises(ValueError):
        sns.check_args(ok, torch.zeros(2, dtype=torch.float64), need_cuda=False)  # b dtype
