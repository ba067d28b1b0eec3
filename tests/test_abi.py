"""CPU-side checks of the C ABI: the library loads, exports every declared entry
point, and its host logic (sphere enumeration, sticks, argument and state
checks) behaves as the header says.  No kernel is launched."""
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from oracle import pw
from workloads import make_workload


def _header_functions():
    text = open(os.path.join(ROOT, "include", "pwlobpcg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pw_[a-zA-Z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_0707_3405_amd as pk
    lib = pk.load_library()
    declared = _header_functions()
    assert len(declared) >= 19
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(pk.EXPORTS)


def test_library_is_gfx950_code_object():
    import paper_0707_3405_amd as pk
    blob = open(pk.library_path(), "rb").read()
    assert b"gfx950" in blob


def test_package_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_0707_3405_amd._binding as b
    monkeypatch.setattr(b, "_LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(b, "_lib", None)
    with pytest.raises(ImportError):
        b.load_library()


def test_fft_sizes_cover_workloads():
    import paper_0707_3405_amd as pk
    sizes = pk.fft_sizes()
    for name in ("gamma_l10", "fcc108_l20", "tiny_nl", "mid_nl", "fcc32_l12"):
        assert make_workload(name).n in sizes


@pytest.mark.parametrize("name", ["gamma_l10", "tiny_nl", "mid_nl", "fcc32_l12", "fcc108_l20"])
def test_host_sphere_matches_oracle(name):
    from paper_0707_3405_amd import Context
    w = make_workload(name)
    c = Context(-1)
    npw = c.init_basis(w.cell, w.kfrac, w.ecut, (w.n,) * 3)
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    assert npw == mil.shape[0]
    assert (c.get_miller() == mil).all()
    assert np.abs(c.get_kinetic() - pw.kinetic(w.cell, w.kfrac, mil)).max() <= 1e-13


def test_host_sphere_general_cell():
    """A non-cubic (but cubic-grid) cell: sphere set equals the oracle's."""
    from paper_0707_3405_amd import Context
    cell = np.array([[7.0, 0.0, 0.0], [1.5, 8.0, 0.0], [0.3, -0.7, 9.0]])
    c = Context(-1)
    c.init_basis(cell, (0.2, -0.1, 0.05), 6.0, (40, 40, 40))
    mil = pw.sphere(cell, (0.2, -0.1, 0.05), 6.0)
    assert (c.get_miller() == mil).all()


def test_argument_and_state_errors():
    from paper_0707_3405_amd import Context, PWError, PW_ERR_ARG, PW_ERR_STATE
    w = make_workload("gamma_l10")
    c = Context(-1)
    with pytest.raises(PWError) as e:
        c.get_miller()
    assert e.value.status == PW_ERR_STATE
    for bad_n in [(24, 24, 25), (25, 25, 25), (8, 8, 8)]:
        with pytest.raises(PWError) as e:
            c.init_basis(w.cell, w.kfrac, w.ecut, bad_n)
        assert e.value.status == PW_ERR_ARG
    with pytest.raises(PWError) as e:
        c.init_basis(w.cell, w.kfrac, -1.0, (24, 24, 24))
    assert e.value.status == PW_ERR_ARG
    c.init_basis(w.cell, w.kfrac, w.ecut, (24, 24, 24))
    # kernels are refused on a host-only context
    with pytest.raises(PWError) as e:
        c.set_local_potential(w.vgrid)
    assert e.value.status == PW_ERR_STATE
    with pytest.raises(PWError) as e:
        c.workspace_size(16, 128)
    assert e.value.status == PW_ERR_ARG
    assert c.workspace_size(16, 16) > 0


def test_band_count_limit_and_density_room():
    """nbands + 3 block <= npw is enforced on the host (every block keeps room
    for [X P W] beside the earlier bands), and the workspace size covers the
    density's N^3 grid however few the bands."""
    from paper_0707_3405_amd import Context, PWError, PW_ERR_ARG
    w = make_workload("gamma_l10")
    c = Context(-1)
    npw = c.init_basis(w.cell, w.kfrac, w.ecut, (w.n,) * 3)
    assert npw == 515
    assert c.workspace_size(npw - 48, 16) > 0
    with pytest.raises(PWError) as e:
        c.workspace_size(npw - 47, 16)
    assert e.value.status == PW_ERR_ARG
    assert c.workspace_size(1, 1) >= w.n ** 3 * 8


def test_binding_refuses_bad_tensors_before_the_library():
    """Blocks of the wrong dtype, too few bands or rows, host memory, a short occupation
    list or a wrong-sized density are refused in Python, before any pointer reaches
    the library (which would read or write past the allocation)."""
    import torch
    from paper_0707_3405_amd import Context, PW_PREC_FP64, PW_PREC_MIXED
    w = make_workload("gamma_l10")
    ctx = Context(-1)
    npw = ctx.init_basis(w.cell, w.kfrac, w.ecut, (w.n,) * 3)
    ok = torch.zeros((4, npw), dtype=torch.complex128)
    cases = [
        (lambda: ctx.apply_H(ok.to(torch.complex64), ok), "complex128"),          # dtype vs prec
        (lambda: ctx.apply_H(ok, ok, prec=PW_PREC_MIXED), "complex64"),
        (lambda: ctx.apply_H(ok, ok, nb=5), "columns"),                            # nb > bands
        (lambda: ctx.apply_H(ok[:, : npw - 1], ok), "rows"),                       # ld < npw
        (lambda: ctx.apply_O(ok, ok[:2]), "columns"),
        (lambda: ctx.apply_H(ok, ok), "cuda"),                                     # host memory
        (lambda: ctx.lobpcg_solve(8, 4, 1e-8, 10, ok), "columns"),
        (lambda: ctx.lobpcg_solve(4, 4, 1e-8, 10, ok.to(torch.complex64)), "complex128"),
        (lambda: ctx.density(ok, [1.0, 1.0], torch.zeros(w.n ** 3, dtype=torch.float64)), "occ"),
        (lambda: ctx.density(ok, [1.0] * 4, torch.zeros(w.n ** 3 - 1, dtype=torch.float64)), "elements"),
        (lambda: ctx.density(ok, [1.0] * 4, torch.zeros(w.n ** 3, dtype=torch.float32)), "float64"),
    ]
    for fn, word in cases:
        with pytest.raises(ValueError, match=word):
            fn()
    ctx.close()
    assert PW_PREC_FP64 == 0


def test_served_worker_failure_releases_its_slot():
    """A request whose solve raises is recorded as failed and frees its footprint and
    slot, so the stream still ends and later requests run (stubbed solve, no GPU)."""
    from paper_0707_3405_amd.serve import Server, footprint
    from paper_0707_3405_amd import PW_PREC_FP64
    from workloads import make_request
    reqs = []
    for i in range(4):
        rw, _ = make_request(i, base_seed=2000, L_range=(8.0, 9.0), ecut_range=(5.0, 6.0))
        reqs.append((0.01 * i, rw, PW_PREC_FP64))
    size = max(footprint(rw, p)[1] for _, rw, p in reqs)
    calls = []

    def stub(rw, prec, device, torch):
        calls.append(rw.name)
        if rw.name == reqs[1][1].name:
            raise RuntimeError("PW_ERR_NUMERIC: planted")
        return {"name": rw.name, "nbands": rw.nbands, "prec": int(prec), "eig": np.zeros(rw.nbands),
                "max_residual": 0.0, "converged": True, "solve_s": 0.0}

    srv = Server(budget_bytes=size, max_active=1, solve=stub)     # one at a time
    results, summary = srv.run(reqs)
    assert sorted(calls) == sorted(r[1].name for r in reqs)
    assert summary["failed"] == 1 and not summary["all_converged"]
    assert results[1]["error"].startswith("RuntimeError")
    assert all(results[i]["error"] is None for i in (0, 2, 3))


def test_radix_split_tuning_is_checked_on_the_host():
    """fft_radix2 must be 0 or a second factor R2 of N = R1 R2 with both factors in
    [2, 16] made of 2, 3, 5; a basis change drops a split the new grid cannot use."""
    from paper_0707_3405_amd import Context, PWError, PW_ERR_ARG
    w = make_workload("gamma_l10")            # N = 24
    ctx = Context(-1)
    ctx.init_basis(w.cell, w.kfrac, w.ecut, (w.n,) * 3)
    for bad in (1, 5, 7, 24, 17):
        with pytest.raises(PWError) as e:
            ctx.set_tuning(fft_radix2=bad)
        assert e.value.status == PW_ERR_ARG
    for ok in (2, 3, 4, 6, 8, 12):
        ctx.set_tuning(fft_radix2=ok)
    ctx.set_tuning(fft_radix2=12)
    w2 = make_workload("mid_nl")              # N = 36: 12 divides, so it stays
    ctx.init_basis(w2.cell, w2.kfrac, w2.ecut, (w2.n,) * 3)
    ctx.set_tuning(fft_radix2=9)              # 36 = 4 x 9
    w3 = make_workload("tiny_nl")             # N = 20: 9 does not divide it: back to the default
    ctx.init_basis(w3.cell, w3.kfrac, w3.ecut, (w3.n,) * 3)
    ctx.set_tuning(fft_radix2=5)
    ctx.close()


def test_apply_batch_argument_checks():
    """pw_apply_H_batch refuses a bad batch before touching a device: no contexts,
    more than 16, a null context, and host-only contexts (no device to run on)."""
    import ctypes
    from paper_0707_3405_amd import Context, PW_ERR_ARG, PW_ERR_STATE
    from workloads import make_workload
    w = make_workload("gamma_l10")
    c = Context(-1)
    c.init_basis(w.cell, w.kfrac, w.ecut, (w.n,) * 3)
    lib = c.lib
    one = (ctypes.c_void_p * 17)(*([c.h.value] * 17))
    ptrs = (ctypes.c_void_p * 17)(*([1] * 17))
    lds = (ctypes.c_int64 * 17)(*([c.npw] * 17))
    assert lib.pw_apply_H_batch(one, 0, ptrs, lds, ptrs, lds, 4, 0) == PW_ERR_ARG
    assert lib.pw_apply_H_batch(one, 17, ptrs, lds, ptrs, lds, 4, 0) == PW_ERR_ARG
    nul = (ctypes.c_void_p * 2)(c.h.value, None)
    assert lib.pw_apply_H_batch(nul, 2, ptrs, lds, ptrs, lds, 4, 0) in (PW_ERR_ARG, PW_ERR_STATE)
    assert lib.pw_apply_H_batch(one, 1, ptrs, lds, ptrs, lds, 4, 0) == PW_ERR_STATE   # host-only
    c.close()
