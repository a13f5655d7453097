"""The workspace-free deflate_project (scratch in a device array inside the
library) against the workspace entry point and against numpy, through the
C ABI: two calls in a row on the same GPU, the second with a smaller input,
and the size limit rejected on the host."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _rand(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def _call_both(n, m, seed):
    import torch
    from paper_0910_2927_amd import _lib
    from tests.gpu_util import torch_dev, announce
    lib = _lib.load()
    dev = torch_dev()
    rng = np.random.default_rng(seed)
    R = _rand(rng, m, n)
    Lv = _rand(rng, m, n)
    F = _rand(rng, m, m)                      # row-major (m, m); the ABI takes column-major
    v = _rand(rng, n)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    Rd, Ld, vd = t(R), t(Lv), t(v)
    Fd = t(F.T)                               # column-major storage of F
    out = {}
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda x: C.c_void_p(x.data_ptr())
    for name in ("workspace", "noalloc"):
        r = torch.empty(n, dtype=torch.complex128, device=dev)
        xp = torch.empty_like(r)
        c = torch.empty(m, dtype=torch.complex128, device=dev)
        announce(f"deflate_project {name} n={n} m={m}")
        if name == "workspace":
            nb = lib.deflate_project_workspace_bytes(m, n)
            ws = torch.empty(nb, dtype=torch.uint8, device=dev)
            st = lib.deflate_project(m, n, p(Rd), p(Ld), p(Fd), p(vd), p(r), p(xp), p(c), p(ws), nb, stream)
        else:
            st = lib.deflate_project_noalloc(m, n, p(Rd), p(Ld), p(Fd), p(vd), p(r), p(xp), p(c), stream)
        _lib.check(st)
        torch.cuda.synchronize()
        out[name] = (r.cpu().numpy(), c.cpu().numpy(), xp.cpu().numpy())
    coeff = Lv.conj() @ v
    ref = (v - R.T @ coeff, coeff, R.T @ (F @ coeff))
    return out, ref


def test_noalloc_matches_workspace_entry_point_twice_shrinking():
    for n, m in ((12 * 4 * 4 * 4 * 6, 24), (12 * 2 * 3 * 2 * 2, 5)):
        out, ref = _call_both(n, m, 1000 + n)
        for a, b_, r_ in zip(out["noalloc"], out["workspace"], ref):
            assert np.array_equal(a, b_)                    # same kernels, same order: identical
            assert np.linalg.norm(a - r_) <= 1e-13 * np.linalg.norm(r_)


def test_noalloc_rejects_sizes_beyond_its_scratch():
    from paper_0910_2927_amd import _lib
    lib = _lib.load()
    n = 12 * 17 ** 4
    st = lib.deflate_project_noalloc(8, n, C.c_void_p(256), C.c_void_p(512), C.c_void_p(768),
                                     C.c_void_p(1 << 40), C.c_void_p(1 << 41), None, C.c_void_p(1 << 42), None)
    assert st == _lib.SK_ERR_ARG
    assert b"workspace-free limit" in lib.sk_last_error()
