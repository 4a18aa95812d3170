"""The library's diagnostic kernels (the counter-calibration copy and the
random-load ceiling): the streaming copy moves exactly its bytes and the
random gather runs on any table of whole words; both reject bad arguments on
the host, before any launch (PM_EINVAL); the profiler times the copy."""
import sys

import pytest

from paper_1411_4942_amd import pathsamp as ps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def test_device_copy_moves_its_bytes():
    for nbytes in (16, 4096, (1 << 20) + 48):
        _say("device_copy", nbytes)
        src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
        dst = torch.zeros_like(src)
        ps.device_copy(dst, src)
        torch.cuda.synchronize()
        assert torch.equal(dst, src), nbytes
    assert ps.lib().pm_device_copy(None, None, 0, None) == ps.PM_OK  # nothing to move


def test_device_copy_rejects_bad_arguments():
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    p, s, L = buf.data_ptr(), torch.cuda.current_stream().cuda_stream, ps.lib()
    assert p % 256 == 0
    assert L.pm_device_copy(p + 1024, p, 40, s) == ps.PM_EINVAL      # not whole 16-byte words
    assert L.pm_device_copy(p + 1028, p, 32, s) == ps.PM_EINVAL      # destination misaligned
    assert L.pm_device_copy(p + 1024, p + 8, 32, s) == ps.PM_EINVAL  # source misaligned
    assert L.pm_device_copy(None, p, 32, s) == ps.PM_EINVAL
    torch.cuda.synchronize()
    assert int(buf.sum()) == 0  # nothing ran


def test_device_gather_runs_and_rejects_bad_tables():
    t = torch.arange(1 << 20, dtype=torch.int32, device="cuda")
    p, s, L = t.data_ptr(), torch.cuda.current_stream().cuda_stream, ps.lib()
    _say("device_gather")
    ps.device_gather(t, 1 << 20, seed=3)
    assert L.pm_device_gather(p, 4, 1000, 1, s) == ps.PM_OK  # a one-word table
    assert L.pm_device_gather(p, 64, 0, 1, s) == ps.PM_OK    # no loads
    torch.cuda.synchronize()
    assert L.pm_device_gather(p, 2, 10, 1, s) == ps.PM_EINVAL      # below one word
    assert L.pm_device_gather(p + 2, 64, 10, 1, s) == ps.PM_EINVAL  # misaligned
    assert L.pm_device_gather(p, 64, -1, 1, s) == ps.PM_EINVAL
    assert L.pm_device_gather(None, 64, 10, 1, s) == ps.PM_EINVAL
    assert torch.equal(t, torch.arange(1 << 20, dtype=torch.int32, device="cuda"))  # read only


def test_profiler_times_the_copy():
    src = torch.ones(1 << 20, dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    try:
        ps.profile_enable(True)
        for _ in range(3):
            ps.device_copy(dst, src)
        got = ps.profile_read()
    finally:
        ps.profile_enable(False)
    assert got["stream_copy"][0] == 3 and got["stream_copy"][1] > 0.0
