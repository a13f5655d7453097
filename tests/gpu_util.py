"""Helpers shared by the GPU tests: move seeded inputs to the device in the
library's layout and bring results back in the canonical layout."""
import numpy as np

import skinputs as si


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def make_op(U, dims, kappa, mu, anti=True, with_c64=False):
    import torch
    from paper_0910_2927_amd import api
    dev = torch_dev()
    links = torch.from_numpy(si.links_soa_from_canonical(U).reshape(-1)).to(dev)
    l64 = links.to(torch.complex64) if with_c64 else None
    return api.WilsonOperator(links, dims, kappa, mu, anti, links64=l64)


def to_dev(vec, V, dtype=None):
    import torch
    t = torch.from_numpy(si.soa_from_canonical(vec, V)).to(torch_dev())
    return t.to(dtype) if dtype is not None else t


def from_dev(t, V):
    return si.canonical_from_soa(t.detach().cpu().numpy().astype(np.complex128), V)


def vecs_to_dev(M, V):
    """Columns of M (n x m, canonical) -> device tensor (m, n) in SoA layout."""
    import torch
    rows = [si.soa_from_canonical(M[:, i], V) for i in range(M.shape[1])]
    return torch.from_numpy(np.ascontiguousarray(np.stack(rows))).to(torch_dev())


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def announce(msg):
    """Name the case before a GPU step (flushed) so a failing run says what ran."""
    print(f"[gpu-case] {msg}", flush=True)
