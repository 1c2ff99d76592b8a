"""The allocation-free geometry backward (mg_geometry_bwd_noalloc) against
mg_geometry_bwd through the C ABI: same result bits, on two calls in a row,
the second with a smaller grid, and sizes beyond the library's fixed scratch
array rejected on the host."""
import ctypes
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PSI_SCALE = json.load(open(os.path.join(ROOT, "tests", "golden", "psi_scale.json")))["scale"]


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_10983_amd import _lib
    return _lib.load()


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _inputs(n, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    psi = torch.from_numpy(PSI_SCALE[str(n)] * W.psi_unit(n)).cuda()
    cbar = torch.randn((6, n, n, n), generator=g, device="cuda", dtype=torch.float64)
    sbar = torch.randn((n, n, n), generator=g, device="cuda", dtype=torch.float64)
    return psi, cbar, sbar


@pytest.mark.parametrize("sizes", [(256, 32), (128, 64)])
def test_noalloc_matches_allocating_entry(lib, sizes):
    from paper_2607_10983_amd import _lib
    for k, n in enumerate(sizes):
        psi, cbar, sbar = _inputs(n, 10 * n + k)
        h = 1.0 / n
        for sb in (sbar, None):
            ref = torch.empty_like(psi)
            out = torch.full_like(psi, float("nan"))
            print(f"geometry_bwd n={n} sqrtgbar={'yes' if sb is not None else 'no'}", flush=True)
            assert lib.mg_geometry_bwd(n, h, _p(psi), _p(cbar), _p(sb), _p(ref), _stream()) == _lib.MG_OK
            assert lib.mg_geometry_bwd_noalloc(n, h, _p(psi), _p(cbar), _p(sb), _p(out), _stream()) == _lib.MG_OK
            torch.cuda.synchronize()
            assert torch.equal(out, ref), float((out - ref).abs().max())


def test_noalloc_rejects_sizes_beyond_scratch(lib):
    from paper_2607_10983_amd import _lib
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    n = 2 * _lib.MG_NOALLOC_MAX_N
    assert lib.mg_geometry_bwd_noalloc(n, 1.0 / n, _p(x), _p(x), None, _p(x), _stream()) == _lib.MG_ERR_INVALID
    assert lib.mg_geometry_bwd_noalloc(48, 1.0 / 48, _p(x), _p(x), None, _p(x), _stream()) == _lib.MG_ERR_INVALID
