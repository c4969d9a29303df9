"""The bandwidth probe runs on the device and leaves its output untouched
for finite input (its store is reached only by a sum no finite input of this
size produces)."""
import pytest

pytestmark = pytest.mark.gpu


def test_read_probe_runs_every_shape(gpu_lib):
    import torch
    sns = gpu_lib
    buf = torch.ones((1 << 24) + 4, dtype=torch.float32, device="cuda")  # ragged tail
    out = torch.zeros(4096, dtype=torch.float32, device="cuda")
    for threads in (256, 512, 1024):
        for unroll in (1, 4):
            for nt in (False, True):
                sns.sns_read_probe(buf, 4096, threads, unroll, nt, out)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(out)) == 0
