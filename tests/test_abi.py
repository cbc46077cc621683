"""The C interface without a GPU: the library loads, exports every entry point
that include/ptrt.h declares, reports the documented velocity tables and
rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from oracle import ptrt as O

P = pytest.importorskip("paper_2602_06686_amd.ptrt")


def _declared():
    src = open(os.path.join(ROOT, "include", "ptrt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ptrt_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = ctypes.CDLL(P.LIB_PATH)
    declared = _declared()
    assert len(declared) >= 28
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(P.EXPORTED) == declared


@pytest.mark.parametrize("lat", [0, 1, 2])
def test_velocity_tables_match_oracle(lat):
    e, w = P.ptrt_velocity_set(lat)
    eo, wo, _ = O.lattice(lat)
    assert (e == eo).all()
    assert np.abs(w - wo).max() < 1e-16


def test_velocity_set_rejects_unknown_lattice():
    assert P._lib.ptrt_velocity_set(7, None, None) == -1


@pytest.mark.parametrize("args,code", [
    ((3, 8, 8, 1, 0.6, 0.25), -1),        # unknown lattice
    ((0, 8, 8, 2, 0.6, 0.25), -1),        # D2Q9 with nz != 1
    ((1, 0, 8, 8, 0.6, 0.25), -1),        # empty lattice
    ((1, 2048, 2048, 1024, 0.6, 0.25), -1),  # 2^32 nodes
    ((0, 8, 8, 1, 0.5, 0.25), -2),        # tau+ = 1/2
    ((0, 8, 8, 1, 0.7, 0.0), -2),         # Lambda = 0
    ((0, 8, 8, 1, float("nan"), 0.25), -2),
])
def test_create_validation(args, code):
    with pytest.raises(P.PtrtError) as ei:
        P.ptrt_create(*args)
    assert ei.value.code == code
    assert P.ptrt_last_error() != "no error"


def test_nonfinite_force_rejected():
    with pytest.raises(P.PtrtError) as ei:
        P.ptrt_create(0, 8, 8, 1, 0.7, 0.25, force=[float("inf"), 0, 0])
    assert ei.value.code == -2


def test_state_errors_without_device():
    h = P.ptrt_create(1, 4, 5, 6, 0.7, 0.25)
    try:
        with pytest.raises(P.PtrtError) as ei:
            P.ptrt_step(h, 1)
        assert ei.value.code == -6               # step before init
        with pytest.raises(P.PtrtError) as ei:
            P.ptrt_step(h, -1)
        assert ei.value.code == -1
        with pytest.raises(P.PtrtError):
            P.ptrt_set_storage(h, 9)
        with pytest.raises(P.PtrtError):
            P.ptrt_set_storage(h, 6)
        assert P.ptrt_get_time(h) == 0
        assert P.ptrt_bytes_per_node(h) == 2 * 19 * 4
    finally:
        P.ptrt_destroy(h)
    assert P._lib.ptrt_destroy(None) == 0


def test_batch_create_validation():
    with pytest.raises(P.PtrtError) as ei:
        P.ptrt_batch_create([{"nx": 8, "ny": 8, "tau_plus": 0.4, "Lambda": 0.25}])
    assert ei.value.code == -2
    assert "instance 0" in P.ptrt_batch_last_error()
    with pytest.raises(P.PtrtError):
        P.ptrt_batch_create([])


def test_forcing_validation_without_device():
    h = P.ptrt_create(0, 8, 8, 1, 0.7, 0.25, force=[1e-5, 0, 0])
    try:
        with pytest.raises(P.PtrtError) as ei:
            P.ptrt_set_forcing(h, 7)
        assert ei.value.code == -1
        P.ptrt_set_forcing(h, "guo")
        P.ptrt_set_forcing(h, "scheme2+g")
        with pytest.raises(P.PtrtError) as ei:
            P.ptrt_set_model(h, "trt-rlb")          # comparison models: default forcing only
        assert ei.value.code == -1
        P.ptrt_set_forcing(h, "scheme2")
    finally:
        P.ptrt_destroy(h)
    assert P.FORCING == {"scheme2": 0, "scheme2+g": 1, "guo": 2}


@pytest.mark.parametrize("lat,nx", [(0, 1 << 29), (1, 240_000_000), (2, 160_000_000)])
def test_rows_beyond_32bit_offsets_rejected(lat, nx):
    """Rows so long that Q * pitch reaches 2^32 elements would wrap the
    kernels' 32-bit in-tile offsets: rejected on the host (no device use)."""
    with pytest.raises(P.PtrtError) as ei:
        P.ptrt_create(lat, nx, 1, 1, 0.7, 0.25)
    assert ei.value.code == -1
    assert "32-bit" in P.ptrt_last_error()
    with pytest.raises(P.PtrtError) as ei:
        P.ptrt_batch_create([{"nx": 1 << 29, "ny": 1, "tau_plus": 0.7, "Lambda": 0.25}])
    assert ei.value.code == -1
    assert "instance 0" in P.ptrt_batch_last_error() and "32-bit" in P.ptrt_batch_last_error()


def test_long_rows_below_the_limit_accepted():
    """9 * 2^28 elements per tile is below 2^32: accepted in every storage
    type (nothing is allocated before init)."""
    h = P.ptrt_create(0, 1 << 28, 1, 1, 0.7, 0.25)
    try:
        for st in (0, 2, 3, 4, 5, 1):
            P.ptrt_set_storage(h, st)
    finally:
        P.ptrt_destroy(h)


def test_divergence_check_arguments_without_device():
    h = P.ptrt_create(1, 8, 8, 8, 0.7, 0.25)
    try:
        with pytest.raises(P.PtrtError) as ei:
            P.ptrt_set_divergence_check(h, -1)
        assert ei.value.code == -1
        P.ptrt_set_divergence_check(h, 0)        # off: nothing to allocate
        assert P.ptrt_divergence_step(h) == -1
    finally:
        P.ptrt_destroy(h)
    assert P._lib.ptrt_divergence_step(None, None) == -1


def test_noalloc_momentum_exchange_rejects_lattices_beyond_its_scratch():
    """The fixed scratch holds 699040 partials of 64 x 4 node blocks: a
    lattice of 1000 x 700 blocks is rejected with a message, before any
    device use; without a completed step a fitting lattice gets
    PTRT_ESTATE."""
    nx, ny = 64 * 1000, 4 * 700
    mask = np.zeros((1, ny, nx), np.uint8)
    mask[0, 0, 0] = 1
    h = P.ptrt_create(0, nx, ny, 1, 0.7, 0.25, solid_mask=mask)
    try:
        with pytest.raises(P.PtrtError) as ei:
            P.ptrt_momentum_exchange_noalloc(h)
        assert ei.value.code == -1 and "scratch" in P.ptrt_last_error(h)
    finally:
        P.ptrt_destroy(h)
    h = P.ptrt_create(0, 64, 64, 1, 0.7, 0.25, solid_mask=mask[:, :64, :64])
    try:
        with pytest.raises(P.PtrtError) as ei:
            P.ptrt_momentum_exchange_noalloc(h)
        assert ei.value.code == -6
    finally:
        P.ptrt_destroy(h)
