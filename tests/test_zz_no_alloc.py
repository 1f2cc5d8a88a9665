"""The allocation-free backward (pdmp_occupancy_bwd_noalloc, for callers that cannot
allocate) against the workspace backward on the same inputs: the same kernels read and
write the static scratch instead of a workspace, so the outputs are the same bits.
Two calls in a row, the second on fewer points, so that the first call's contents of
the shared scratch cannot leak into the second; then a size beyond the scratch is
refused before any launch."""
import numpy as np
import pytest

import paper_2108_11775_amd as P
from paper_2108_11775_amd import _lib, configs as K, inputs as I

from helpers import arm_scene, dev, gpu_occ, host, require_gpu, ws_scene

pytestmark = pytest.mark.gpu


def _pair(occ, x, g, s_fwd):
    import torch
    gw_ref, gx_ref = P.occupancy_bwd(occ, x, g, s_fwd=s_fwd)
    n = int(x.shape[1])
    gw = torch.full((occ.n_hinges + 1,), float("nan"), dtype=torch.float32, device=x.device)
    gx = torch.full((occ.dim, n), float("nan"), dtype=torch.float32, device=x.device)
    P.occupancy_bwd_noalloc(occ, x, g, s_fwd=s_fwd, grad_w=gw, grad_x=gx)
    P.sync()
    assert np.array_equal(host(gw), host(gw_ref))
    assert np.array_equal(host(gx), host(gx_ref))


def test_noalloc_backward_matches_workspace_backward():
    require_gpu()
    sc = arm_scene()
    occ3 = gpu_occ(sc["h"], sc["wb"], sc["ell"], (16, 16, 16))
    n1, n2 = K.C4.n_points, 30001
    x1 = I.uniform_points(K.C4.cfg_id, K.STREAM_FIT, 3, n1, -1, 1)
    g1 = (I.rng(4, 21).normal(size=n1) / n1).astype(np.float32)
    # first call: the 3-D grid at the fit's 2^20 points, chained through sigma'(s)
    s1 = host(P.occupancy_eval(occ3, dev(x1))[1])
    _pair(occ3, dev(x1), dev(g1), dev(s1))
    # second call, fewer points and the logit form (no chain)
    x2 = np.ascontiguousarray(x1[:, :n2])
    g2 = (I.rng(4, 22).normal(size=n2) / n2).astype(np.float32)
    _pair(occ3, dev(x2), dev(g2), None)
    # a 2-D pairwise occupancy on the same scratch
    cfg = K.C1
    s2 = ws_scene(cfg)
    occ2 = gpu_occ(s2["h"], s2["wb"], s2["ell"])
    x3 = I.uniform_points(cfg.cfg_id, K.STREAM_EVAL, 2, 777, cfg.lo, cfg.hi)
    _pair(occ2, dev(x3), dev(np.ones(777, np.float32)), None)


def test_noalloc_backward_refuses_sizes_beyond_the_scratch():
    require_gpu()
    lib = _lib.load()
    n = 1 << 23  # 2^23 points at 4096 hinges need more than the 32 MiB scratch
    assert lib.pdmp_bwd_workspace_size(3, 4096, n) > 32 << 20
    sc = arm_scene()
    occ3 = gpu_occ(sc["h"], sc["wb"], sc["ell"], (16, 16, 16))
    import ctypes as C
    o = occ3.c_struct()
    st = lib.pdmp_occupancy_bwd_noalloc(C.byref(o), C.c_void_p(16), n, C.c_void_p(16), None,
                                        C.c_void_p(16), None, None)
    assert st == _lib.PDMP_ENOMEM and b"32" in lib.pdmp_last_error()
