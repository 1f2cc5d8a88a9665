"""CPU checks of the C ABI: the library loads, exports every declared symbol, and
rejects invalid arguments on the host before anything is launched."""
import ctypes as C
import re

import pytest

from paper_2108_11775_amd import _lib


def _declared():
    src = open(_lib.HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pdmp_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    names = _declared()
    assert "pdmp_morph_samples" in names and "pdmp_fk_body_points" in names
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.pdmp_abi_version() == 1


def test_invalid_arguments_rejected_before_launch():
    lib = _lib.load()
    E = _lib.PDMP_EINVAL
    assert lib.pdmp_occupancy_eval(None, None, 1, None, None, None) == E
    occ = _lib.pdmp_occupancy(4, 8, 16, 16, 0.5)
    assert lib.pdmp_occupancy_eval(C.byref(occ), None, 1, None, None, None) == E
    assert b"dim" in lib.pdmp_last_error()
    occ = _lib.pdmp_occupancy(2, 8, 16, 16, -1.0)
    assert lib.pdmp_occupancy_grad(C.byref(occ), None, 1, None, None, None) == E
    occ = _lib.pdmp_occupancy(2, 0, 16, 16, 0.5)
    assert lib.pdmp_morph_samples(C.byref(occ), None, None, None, 1, 1, 0.1, None) == E
    occ = _lib.pdmp_occupancy(2, 8, 16, 16, 0.5)
    assert lib.pdmp_morph_samples(C.byref(occ), None, None, None, 1, -1, 0.1, None) == E
    assert lib.pdmp_morph_samples(C.byref(occ), None, None, None, 1, 3, float("nan"), None) == E
    assert lib.pdmp_morph_samples(C.byref(occ), None, None, None, -5, 3, 0.1, None) == E
    # the recording morph: traj and its stride are checked before anything else
    assert lib.pdmp_morph_trajectory(C.byref(occ), None, None, None, 4, 3, 0.1, None, 1,
                                     None) == E
    assert lib.pdmp_morph_trajectory(C.byref(occ), None, None, None, 4, 3, 0.1, C.c_void_p(16),
                                     0, None) == E
    assert b"traj_stride" in lib.pdmp_last_error()
    # a 2-D occupancy cannot drive an arm
    arm = _lib.pdmp_arm()
    arm.n_dof, arm.pts_per_link = 7, 8
    assert lib.pdmp_morph_samples(C.byref(occ), C.byref(arm), None, None, 4, 3, 0.1, None) == E
    arm.n_dof = 9
    assert lib.pdmp_fk_body_points(C.byref(arm), None, 4, None, None) == E
    # weighted MLP backward: the weight is checked on the host (the pointers below are
    # never dereferenced: the call returns before any launch)
    fake = C.c_void_p(256)
    mlp = _lib.pdmp_mlp(7, 64, 2, fake, fake)
    for bad in (-1.0, float("nan"), float("inf")):
        assert lib.pdmp_mlp_backward_weighted(C.byref(mlp), fake, fake, 16, None, bad, fake,
                                              fake, None, fake, 1 << 30, None) == E
        assert b"hard_weight" in lib.pdmp_last_error()
    assert lib.pdmp_mlp_backward_weighted(C.byref(mlp), fake, fake, 0, None, 2.0, fake, fake,
                                          None, fake, 1 << 30, None) == E
    arm.n_dof, arm.pts_per_link = 7, 12
    occ3 = _lib.pdmp_occupancy(3, 8, 16, 16, 0.5)
    assert (lib.pdmp_morph_samples(C.byref(occ3), C.byref(arm), None, None, 4, 3, 0.1, None)
            == _lib.PDMP_EUNSUPPORTED)
    lo = (C.c_float * 2)(0.0, 1.0)
    hi = (C.c_float * 2)(1.0, 0.0)
    assert lib.pdmp_uniform_samples(1, 0, lo, hi, 2, 10, None, None) == E
    assert lib.pdmp_uniform_samples(1, 0, lo, lo, 17, 10, None, None) == E


def test_empty_batches_are_no_ops_without_a_device():
    lib = _lib.load()
    occ = _lib.pdmp_occupancy(2, 8, 16, 16, 0.5)
    assert lib.pdmp_occupancy_eval(C.byref(occ), None, 0, None, None, None) == 0
    assert lib.pdmp_morph_samples(C.byref(occ), None, None, None, 0, 5, 0.1, None) == 0
    lo = (C.c_float * 1)(0.0)
    assert lib.pdmp_uniform_samples(1, 0, lo, lo, 1, 0, None, None) == 0


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    import paper_2108_11775_amd as P
    occ = P.Occupancy(torch.zeros(2, 4), torch.zeros(5), 0.5)
    with pytest.raises(TypeError):
        P.occupancy_eval(occ, torch.zeros(2, 3))


def test_tanh_network_shapes_checked_on_the_host():
    lib = _lib.load()
    net = _lib.pdmp_tanh_net(2, 64, 3, None)
    assert lib.pdmp_tanh_num_params(C.byref(net)) == 64 * 2 + 64 + 2 * (64 * 64 + 64) + 64 + 1
    for bad in [(4, 8, 2), (2, 65, 2), (2, 0, 2), (3, 8, 0), (3, 8, 5)]:
        b = _lib.pdmp_tanh_net(*bad, None)
        assert lib.pdmp_tanh_num_params(C.byref(b)) == -1
        assert lib.pdmp_tanh_occupancy_eval(C.byref(b), None, 1, None, None, None) == \
            _lib.PDMP_EINVAL
    assert lib.pdmp_tanh_occupancy_grad(C.byref(net), None, 1, None, None, None) == \
        _lib.PDMP_EINVAL  # params NULL
    fake = _lib.pdmp_tanh_net(2, 8, 1, C.c_void_p(16))
    assert lib.pdmp_tanh_morph_samples(C.byref(fake), None, None, 1, -1, 0.1, None) == \
        _lib.PDMP_EINVAL
    assert lib.pdmp_tanh_morph_samples(C.byref(fake), None, None, 0, 3, 0.1, None) == 0
    # the forward scheme query: the network and the out-pointer are checked first
    v = C.c_int32(-1)
    assert lib.pdmp_tanh_split_scheme(None, C.byref(v), None) == _lib.PDMP_EINVAL
    assert lib.pdmp_tanh_split_scheme(C.byref(net), C.byref(v), None) == _lib.PDMP_EINVAL
    assert lib.pdmp_tanh_split_scheme(C.byref(fake), None, None) == _lib.PDMP_EINVAL
    assert b"scheme" in lib.pdmp_last_error()
    import paper_2108_11775_amd as P
    with pytest.raises(ValueError):
        P.TanhNet(2, 100, 2, None)
