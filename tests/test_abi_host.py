"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/ohm.h declares, the header is valid C, and argument
validation answers without touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2206_06079_amd as ohm
from paper_2206_06079_amd import _lib
from workloads import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ohm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:ohm_status|const char\*)\s+(ohm_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_lib.EXPORTS)


def test_header_compiles_as_c():
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", HEADER], check=True)


def test_struct_layouts_match_header(tmp_path):
    src = '#include "ohm.h"\n#include <stdio.h>\n#include <stddef.h>\nint main(void){printf("%zu %zu %zu %zu\\n", sizeof(ohm_params), sizeof(ohm_map_stats), sizeof(ohm_scan_set), sizeof(ohm_batch_tuning)); return 0;}\n'
    exe = str(tmp_path / "abi_sizes")
    subprocess.run(["gcc", "-x", "c", "-", "-I", os.path.join(ROOT, "include"), "-o", exe], input=src.encode(), check=True)
    out = subprocess.run([exe], capture_output=True, check=True).stdout.split()
    sizes = [int(x) for x in out]
    assert sizes == [ctypes.sizeof(_lib.OhmParams), ctypes.sizeof(_lib.OhmStats), ctypes.sizeof(_lib.ScanSet),
                     ctypes.sizeof(_lib.BatchTuning)]


def _size(mp, cap=16, layers=1):
    lib = _lib.load()
    p = _lib.make_params(mp)
    sz = ctypes.c_size_t(0)
    return lib.ohm_map_workspace_size(ctypes.byref(p), cap, layers, ctypes.byref(sz)), sz.value


def test_workspace_size_and_validation():
    mp, _ = scenes.config0()
    st, bytes_ = _size(mp, 343)
    assert st == _lib.OHM_OK
    # 343 regions x 32^3 voxels x (4 B occupancy + 16 B accumulators: two f32
    # slots, which a weighted scan uses as one slot of int64 sums) plus tables
    assert 343 * 32768 * 20 <= bytes_ < 343 * 32768 * 20 + (1 << 22)
    st_ndt, bytes_ndt = _size(mp, 343, _lib.LAYER_NDT | _lib.LAYER_ADJOINT)
    assert st_ndt == _lib.OHM_OK and bytes_ndt > bytes_
    bad = [
        mp.replace(voxel_size=0.0),
        mp.replace(key_max=(0, 200, 200)),
        mp.replace(l_min=1.0, l_max=0.5),
        mp.replace(l_init=9.0),
        mp.replace(fixed_bits=4),
        mp.replace(mode=7),
        mp.replace(sensor_noise=0.0),
        mp.replace(adaptation_rate=1.5),
        mp.replace(l_hit=float("nan")),
    ]
    for b in bad:
        assert _size(b)[0] == _lib.OHM_E_INVALID_ARG, b
    assert _size(mp, 0)[0] == _lib.OHM_E_INVALID_ARG
    assert _size(mp, 70000)[0] == _lib.OHM_E_INVALID_ARG
    # region size other than 32^3 is reported as unsupported
    p = _lib.make_params(mp)
    p.region_log2 = 4
    sz = ctypes.c_size_t()
    assert _lib.load().ohm_map_workspace_size(ctypes.byref(p), 8, 1, ctypes.byref(sz)) == _lib.OHM_E_UNSUPPORTED


def test_scan_group_slots_in_the_layer_mask():
    """OHM_LAYER_SCAN_GROUPS holds G accumulator slots of 256 KiB per region
    of capacity (default G = 8, OHM_SCAN_GROUP_SLOTS(n) for 1..64), at least
    the two every map has; slot bits without the layer, or more than 64
    slots, are rejected."""
    mp, _ = scenes.config0()
    slot = 343 * 32768 * 8
    st, plain = _size(mp, 343)
    assert st == _lib.OHM_OK
    g = _lib.LAYER_SCAN_GROUPS
    for layers, slots in ((g, 8), (g | ohm.scan_group_slots(8), 8), (g | ohm.scan_group_slots(1), 1),
                          (g | ohm.scan_group_slots(16), 16), (g | ohm.scan_group_slots(64), 64)):
        st, b = _size(mp, 343, layers)
        assert st == _lib.OHM_OK, layers
        assert b - plain == (max(slots, 2) - 2) * slot, (layers, b - plain)
    for layers in (ohm.scan_group_slots(8), g | ohm.scan_group_slots(65), g | ohm.scan_group_slots(255)):
        assert _size(mp, 343, layers)[0] == _lib.OHM_E_INVALID_ARG, layers


def test_create_without_device_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    mp, _ = scenes.config0()
    lib = _lib.load()
    p = _lib.make_params(mp)
    st, n = _size(mp, 8)
    h = ctypes.c_void_p()
    # a (fake, never dereferenced) aligned pointer: creation must stop at the device check
    assert lib.ohm_map_create(ctypes.byref(p), 8, 1, ctypes.c_void_p(1 << 20), n, None, ctypes.byref(h)) == \
        _lib.OHM_E_NO_DEVICE
    assert not h.value
    # misaligned workspace and short workspace are argument errors
    assert lib.ohm_map_create(ctypes.byref(p), 8, 1, ctypes.c_void_p(3), n, None, ctypes.byref(h)) == \
        _lib.OHM_E_INVALID_ARG
    assert lib.ohm_map_create(ctypes.byref(p), 8, 1, ctypes.c_void_p(1 << 20), n - 1, None, ctypes.byref(h)) == \
        _lib.OHM_E_WORKSPACE_TOO_SMALL


def test_null_handles_are_rejected():
    lib = _lib.load()
    assert lib.ohm_map_destroy(None) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_map_reset(None, None) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_integrate_rays(None, None, None, None, 0, None, None) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_ndt_integrate(None, None, None, None, 0, None, None) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_batch_run(None, None) == _lib.OHM_E_INVALID_ARG
    st = _lib.OhmStats()
    assert lib.ohm_map_sync_status(None, None, ctypes.byref(st)) == _lib.OHM_E_INVALID_ARG
    assert _lib.status_string(_lib.OHM_E_NO_DEVICE) == "no HIP device"


def test_ray_order_scratch_arguments():
    lib = _lib.load()
    sz = ctypes.c_size_t(0)
    assert lib.ohm_ray_order_scratch_size(0, ctypes.byref(sz)) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_ray_order_scratch_size(131072, ctypes.byref(sz)) == _lib.OHM_OK
    # 512 strips x 256 elevation bins, plus one permutation entry per ray, 4 bytes each
    assert sz.value >= 4 * (512 * 256 + 131072)
    assert lib.ohm_map_set_ray_order(None, None, 0, 0) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_map_set_scan_layout(None, 64) == _lib.OHM_E_INVALID_ARG


def test_product_never_imports_oracle():
    """The HIP package must not reach the CPU oracle (no fallback path)."""
    pkg = os.path.join(ROOT, "paper_2206_06079_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", text).lower() or f == "build.py", f


def test_probe_arguments_are_validated():
    """Both measurement probes reject bad arguments before any device call."""
    lib = _lib.load()
    rate = ctypes.c_double(0.0)
    big, fake = 64 << 20, ctypes.c_void_p(1 << 20)  # never dereferenced: rejected first
    # stream probe: null buffers, unaligned buffers, too small, not a multiple of 16, unknown flags
    assert lib.ohm_probe_stream_rate(None, fake, big, 0, ctypes.byref(rate), None) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_probe_stream_rate(fake, None, big, 0, ctypes.byref(rate), None) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_probe_stream_rate(ctypes.c_void_p((1 << 20) + 8), fake, big, 0, ctypes.byref(rate),
                                     None) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_probe_stream_rate(fake, fake, 1 << 20, 0, ctypes.byref(rate), None) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_probe_stream_rate(fake, fake, big + 8, 0, ctypes.byref(rate), None) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_probe_stream_rate(fake, fake, big, _lib.PROBE_SEQUENTIAL, ctypes.byref(rate),
                                     None) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_probe_stream_rate(fake, fake, big, 0, None, None) == _lib.OHM_E_INVALID_ARG
    # atomic probe: null buffer, too small, conflicting operations
    assert lib.ohm_probe_atomic_rate(None, big, 0, ctypes.byref(rate), None) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_probe_atomic_rate(fake, 2, 0, ctypes.byref(rate), None) == _lib.OHM_E_INVALID_ARG
    assert lib.ohm_probe_atomic_rate(fake, big, _lib.PROBE_F32_CAS | _lib.PROBE_U64_ADD, ctypes.byref(rate),
                                     None) == _lib.OHM_E_INVALID_ARG
