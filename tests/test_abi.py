"""CPU checks of the C ABI: the library loads, exports every declared symbol, and validates
parameters before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2609_28679_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(lbm_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2609_28679_amd import build
        build.build()
    return binding.load()


def test_library_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.SIGNATURES), "binding and header disagree"


def test_default_params_and_workspace_size(lib):
    p = binding.LbmParams()
    lib.lbm_default_params(ctypes.byref(p))
    assert (p.lattice, p.model, p.storage, p.nx, p.ny, p.nz) == (0, 0, 0, 64, 64, 1)
    assert p.tau == 0.8 and p.fp16_scale_log2 == 16
    assert p.streaming == 0  # automatic layout
    nbytes = ctypes.c_size_t(0)
    p.streaming = binding.STREAMINGS["two"]
    assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)) == 0
    # two population buffers of 9 float32 planes at least
    assert nbytes.value >= 2 * 9 * 64 * 64 * 4
    p.storage = binding.STORAGES["fp64"]
    big = ctypes.c_size_t(0)
    assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(big)) == 0
    assert big.value > nbytes.value


@pytest.mark.parametrize("field,value", [("tau", 0.5), ("tau", float("nan")), ("nx", 0),
                                          ("nz", 2), ("lattice", 7), ("wall_y", 2),
                                          ("diag_every", -1), ("streaming", 3),
                                          ("streaming", -1)])
def test_invalid_params_rejected(lib, field, value):
    p = binding.LbmParams()
    lib.lbm_default_params(ctypes.byref(p))
    setattr(p, field, value)
    nbytes = ctypes.c_size_t(0)
    assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)) == binding.LBM_EINVAL
    assert lib.lbm_last_error(None)


def _create(lib, rho, u, **kw):
    p = binding.LbmParams()
    lib.lbm_default_params(ctypes.byref(p))
    p.ny, p.nx = rho.shape
    for k, v in kw.items():
        setattr(p, k, v)
    ctx = ctypes.c_void_p()
    rc = lib.lbm_create(ctypes.byref(p), rho.ctypes.data_as(binding._D),
                        u.ctypes.data_as(binding._D), None, ctypes.byref(ctx))
    return rc, ctx


def test_create_rejects_inadmissible_initial_state_before_device_work(lib):
    rho = np.ones((4, 5))
    u = np.zeros((2, 4, 5))
    u[0, 1, 2] = 0.9  # theta + u^2 > 1: negative rest factor
    rc, ctx = _create(lib, rho, u)
    assert rc == binding.LBM_EINVAL and not ctx.value
    assert b"product-form" in lib.lbm_last_error(None)
    u[0, 1, 2] = 0.0
    rho[3, 4] = np.nan
    rc, ctx = _create(lib, rho, u)
    assert rc == binding.LBM_EINVAL and not ctx.value


def test_null_context_is_a_state_error(lib):
    assert lib.lbm_step(None, 1) == binding.LBM_ESTATE
    assert lib.lbm_set_force(None, (ctypes.c_double * 3)(0.0, 0.0, 0.0)) == binding.LBM_ESTATE
    assert lib.lbm_set_heat_source(None, 0.0) == binding.LBM_ESTATE
    lib.lbm_destroy(None)  # NULL-safe


def _workspace(lib, **kw):
    p = binding.LbmParams()
    lib.lbm_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    n = ctypes.c_size_t(0)
    rc = lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n))
    return rc, n.value


def test_one_buffer_layout_halves_population_memory(lib):
    one = binding.STREAMINGS["one"]
    two = binding.STREAMINGS["two"]
    auto = binding.STREAMINGS["auto"]
    for storage, elem in (("fp32", 4), ("fp64", 8)):
        st = binding.STORAGES[storage]
        rc1, b1 = _workspace(lib, nx=1024, ny=1024, storage=st, streaming=one)
        rc2, b2 = _workspace(lib, nx=1024, ny=1024, storage=st, streaming=two)
        assert rc1 == rc2 == 0
        assert b2 - b1 >= 9 * 1024 * 1024 * elem
    # D3Q27 too
    rc3, b3 = _workspace(lib, lattice=1, nx=64, ny=64, nz=64, streaming=one)
    rc4, b4 = _workspace(lib, lattice=1, nx=64, ny=64, nz=64, streaming=two)
    assert rc3 == rc4 == 0 and b4 - b3 >= 27 * 64 ** 3 * 4
    # automatic choice: one buffer while it stays within 384 MiB, two beyond
    _, small_auto = _workspace(lib, nx=2048, ny=2048, streaming=auto)
    _, small_one = _workspace(lib, nx=2048, ny=2048, streaming=one)
    _, big_auto = _workspace(lib, nx=4096, ny=4096, streaming=auto)
    _, big_two = _workspace(lib, nx=4096, ny=4096, streaming=two)
    assert small_auto == small_one and big_auto == big_two


@pytest.mark.parametrize("kw", [dict(model=1), dict(storage=1), dict(storage=2),
                                dict(collision=1)])
def test_one_buffer_layout_rejected_where_unsupported(lib, kw):
    rc, _ = _workspace(lib, streaming=binding.STREAMINGS["one"], **kw)
    assert rc == binding.LBM_EINVAL
    assert b"one-buffer" in lib.lbm_last_error(None)
    rc, _ = _workspace(lib, streaming=binding.STREAMINGS["auto"], **kw)
    assert rc == 0


@pytest.mark.parametrize("kw", [dict(storage=1), dict(storage=2), dict(model=1, storage=1),
                                dict(collision=1), dict(force_z=1e-6),
                                dict(force_x=float("nan")), dict(force_y=float("inf")),
                                dict(heat=1e-6), dict(model=1, storage=2, heat=1e-6, force_x=0.0),
                                dict(model=1, heat=float("nan"), force_x=0.0)])
def test_sources_rejected_where_unsupported(lib, kw):
    kw = dict(kw)
    force = [kw.pop("force_x", 1e-6), kw.pop("force_y", 0.0), kw.pop("force_z", 0.0)]
    heat = kw.pop("heat", 0.0)
    p = binding.LbmParams()
    lib.lbm_default_params(ctypes.byref(p))
    assert list(p.force) == [0.0, 0.0, 0.0]  # default: no force
    for k, v in kw.items():
        setattr(p, k, v)
    for a in range(3):
        p.force[a] = force[a]
    p.heat_source = heat
    n = ctypes.c_size_t(0)
    assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == binding.LBM_EINVAL
    assert b"force" in lib.lbm_last_error(None) or b"heat_source" in lib.lbm_last_error(None)


@pytest.mark.parametrize("lattice, model, nz, force, heat", [
    (0, 0, 1, (1e-6, -2e-6, 0.0), 0.0), (1, 0, 8, (0.0, 1e-6, 3e-6), 0.0),
    (0, 1, 1, (1e-6, -2e-6, 0.0), 0.0), (0, 1, 1, (0.0, 0.0, 0.0), 1e-5),
    (0, 1, 1, (1e-6, 0.0, 0.0), -1e-5)])
def test_sources_accepted(lib, lattice, model, nz, force, heat):
    for storage in (0, 3):  # float32, float64
        for streaming in ((1, 2) if model == 0 else (0,)):
            p = binding.LbmParams()
            lib.lbm_default_params(ctypes.byref(p))
            assert p.heat_source == 0.0
            p.lattice, p.model, p.nx, p.ny, p.nz = lattice, model, 8, 8, nz
            p.storage, p.streaming = storage, streaming
            for a in range(3):
                p.force[a] = force[a]
            p.heat_source = heat
            n = ctypes.c_size_t(0)
            assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0


@pytest.mark.parametrize("kw", [dict(prandtl=0.0), dict(prandtl=float("nan")),
                                dict(eta_over_mu=float("inf")), dict(prandtl=2.0),
                                dict(eta_over_mu=1.0), dict(model=1, storage=1, prandtl=2.0),
                                dict(model=1, storage=2, eta_over_mu=0.0)])
def test_transport_parameters_validated(lib, kw):
    rc, _ = _workspace(lib, **kw)
    assert rc == binding.LBM_EINVAL
    assert b"prandtl" in lib.lbm_last_error(None) or b"eta_over_mu" in lib.lbm_last_error(None)


def test_transport_parameters_accepted_for_the_thermal_model(lib):
    p = binding.LbmParams()
    lib.lbm_default_params(ctypes.byref(p))
    assert p.prandtl == 1.0 and p.eta_over_mu < 0
    for storage in (0, 3):
        rc, _ = _workspace(lib, model=1, storage=storage, prandtl=0.71, eta_over_mu=0.0)
        assert rc == 0


def _neq_params(lib, **kw):
    p = binding.LbmParams()
    lib.lbm_default_params(ctypes.byref(p))
    p.model, p.wall_y, p.ny = 1, 2, 16
    p.wall_T[0], p.wall_T[1] = 1.0, 1.1
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("kw", [dict(model=0), dict(storage=1), dict(lattice=1, nz=4, storage=2),
                                dict(ny=2), dict(lattice=1, nz=4, ny=2), dict(wall_density=2),
                                dict(heat_source=1e-5), dict(lattice=1, nz=4, heat_source=1e-5)])
def test_neq_walls_rejected_where_unsupported(lib, kw):
    p = _neq_params(lib, **kw)
    n = ctypes.c_size_t(0)
    assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == binding.LBM_EINVAL


def test_neq_walls_validate_wall_state(lib):
    n = ctypes.c_size_t(0)
    p = _neq_params(lib)
    assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
    # D3Q27: the boundary planes (2 x 54 of nz x pitch elements) add to the workspace
    n3, n3w = ctypes.c_size_t(0), ctypes.c_size_t(0)
    p3 = _neq_params(lib, lattice=1, nz=4)
    assert lib.lbm_workspace_size(ctypes.byref(p3), ctypes.byref(n3w)) == 0
    p3.wall_y = 1
    assert lib.lbm_workspace_size(ctypes.byref(p3), ctypes.byref(n3)) == 0
    assert n3w.value - n3.value >= 108 * 4 * p3.nx * 4
    p.wall_T[1] = 0.0
    assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == binding.LBM_EINVAL
    p = _neq_params(lib)
    p.wall_u[1][1] = 0.01  # normal wall velocity
    assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == binding.LBM_EINVAL
    p = _neq_params(lib)
    p.wall_u[1][0] = 0.9  # inadmissible product-form factors at the wall
    assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == binding.LBM_EINVAL
    p = _neq_params(lib)
    p.wall_u[0][2] = 0.02  # a z velocity: D3Q27 only
    assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == binding.LBM_EINVAL
    p = _neq_params(lib, lattice=1, nz=4)
    p.wall_u[0][2] = 0.02
    assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
    p.wall_u[0][2] = 0.9
    assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == binding.LBM_EINVAL


@pytest.mark.parametrize("kw", [dict(eos=2), dict(eos=1),
                                dict(eos=1, model=1, storage=1),
                                dict(eos=1, model=1, vdw_a=-1.0),
                                dict(eos=1, model=1, vdw_b=float("nan"))])
def test_van_der_waals_rejected_where_unsupported(lib, kw):
    rc, _ = _workspace(lib, **kw)
    assert rc == binding.LBM_EINVAL


def test_van_der_waals_accepted_for_the_thermal_model(lib):
    for storage in (0, 3):
        rc, _ = _workspace(lib, eos=1, model=1, storage=storage, vdw_a=0.27, vdw_b=0.2)
        assert rc == 0
        rc, _ = _workspace(lib, eos=1, model=1, lattice=1, nz=4, storage=storage, vdw_a=0.27,
                           vdw_b=0.2)
        assert rc == 0


def test_van_der_waals_neq_walls_need_supercritical_wall_isotherms(lib):
    # the pressure-continued wall density solves P(rho_B, T_W) = P_N on the wall isotherm,
    # which has one root only above T_cr = 8 a / (27 b R) = 1.2 here
    n = ctypes.c_size_t(0)
    for lattice, nz in ((0, 1), (1, 4)):
        p = _neq_params(lib, eos=1, vdw_a=0.27, vdw_b=0.2, lattice=lattice, nz=nz)
        p.wall_T[0], p.wall_T[1] = 1.4, 1.45
        assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
        p.wall_T[0] = 1.1  # subcritical wall
        assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == binding.LBM_EINVAL
        p.wall_density = 1  # the literal density needs no root
        assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
        p.wall_density, p.vdw_b, p.wall_T[0] = 0, 0.0, 1.4  # b = 0: no supercritical isotherm
        assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == binding.LBM_EINVAL


@pytest.mark.parametrize("lattice,model,storage,collision,wall_y,nz", [
    (0, 0, 0, 0, 0, 1), (0, 0, 3, 0, 1, 1), (0, 0, 1, 0, 0, 1), (0, 0, 2, 0, 1, 1),
    (0, 0, 0, 1, 0, 1), (0, 0, 0, 1, 1, 1), (0, 1, 0, 0, 1, 1), (0, 1, 3, 0, 2, 1),
    (0, 1, 1, 0, 1, 1), (1, 0, 0, 0, 0, 5), (1, 0, 3, 0, 1, 3), (1, 1, 0, 0, 2, 3),
    (1, 1, 3, 0, 0, 7)])
def test_workspace_regions_are_256_byte_aligned(lib, lattice, model, storage, collision, wall_y,
                                                nz):
    # every region of the workspace (populations, diagnostics partials, history, read-out,
    # the surrogate's 64-bit atomic counters and weights, derivative fields, wall rows) starts
    # on a 256-byte boundary: lbm_workspace_size refuses a plan where one does not, so a
    # successful size over ragged shapes and every configuration is the check
    for nx, ny in ((3, 3), (37, 5), (100, 17), (257, 3), (1000, 33)):
        p = _neq_params(lib, lattice=lattice, model=model, storage=storage, collision=collision,
                        wall_y=wall_y, nx=nx, ny=ny, nz=nz)
        for streaming in (0, 1, 2) if model == 0 and collision == 0 and storage in (0, 3) else (0,):
            p.streaming = streaming
            n = ctypes.c_size_t(0)
            assert lib.lbm_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0, (nx, ny)
            assert n.value % 256 == 0


def test_mlp_gradient_batch_limit_checked_before_state(lib):
    # at most 2^20 samples per gradient call (the partials take 22 KiB per 64 samples)
    f = ctypes.c_float(0.0)
    assert lib.lbm_mlp_grad(None, None, None, (1 << 20) + 1, None, ctypes.byref(f)) == binding.LBM_EINVAL
    assert lib.lbm_mlp_grad(None, None, None, 0, None, ctypes.byref(f)) == binding.LBM_EINVAL
    assert lib.lbm_mlp_grad(None, None, None, 1 << 20, None, ctypes.byref(f)) == binding.LBM_ESTATE

