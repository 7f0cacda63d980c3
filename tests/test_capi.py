"""The C-ABI library loads, exports every symbol include/fdtbx.h declares, and
rejects bad arguments on the host before any launch (no GPU needed)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdtbx.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fdtbx_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2608_23245_amd import binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    return B.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "fdtbx_profile_pattern" in names and len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_2608_23245_amd import binding as B
    assert set(declared()) == set(B.exported_symbols())


def test_host_argument_checks(lib):
    from paper_2608_23245_amd import binding as B
    cell = B.Cell(10, 10, 20, math.pi / 2, math.pi / 2, math.pi / 2)
    cap = ctypes.c_int64(0)
    assert lib.fdtbx_hkl_capacity(ctypes.byref(cell), 4.0, ctypes.byref(cap)) == 0
    assert cap.value == (2 * 3 + 1) * (2 * 3 + 1) * (2 * 6 + 1)
    assert lib.fdtbx_hkl_capacity(ctypes.byref(cell), 0.0, ctypes.byref(cap)) == -1
    assert lib.fdtbx_hkl_capacity(ctypes.byref(cell), float("nan"), ctypes.byref(cap)) == -1
    bad = B.Cell(10, 10, 20, 0.1, 0.1, 3.0)   # angles that span no parallelepiped
    assert lib.fdtbx_hkl_capacity(ctypes.byref(bad), 4.0, ctypes.byref(cap)) == -2
    neg = B.Cell(-1, 10, 20, 1.5, 1.5, 1.5)
    assert lib.fdtbx_hkl_capacity(ctypes.byref(neg), 4.0, ctypes.byref(cap)) == -2
    # null pointers and sizes are rejected before any device work
    assert lib.fdtbx_enumerate_hkl(ctypes.byref(cell), 4.0, 30.0, None, None, 10, None, None, 0, None) == -1
    assert lib.fdtbx_enumerate_hkl(ctypes.byref(cell), 4.0, 3.0, None, ctypes.c_void_p(8), 10 ** 6, ctypes.c_void_p(8),
                                   ctypes.c_void_p(8), 10 ** 6, None) == -1  # d_max below d_min
    assert lib.fdtbx_enumerate_hkl(ctypes.byref(cell), 4.0, 30.0, None, ctypes.c_void_p(8), 5, ctypes.c_void_p(8),
                                   ctypes.c_void_p(8), 10 ** 6, None) == -3  # capacity below the box
    msg = lib.fdtbx_error_string(-3).decode()
    assert "capacity" in msg
    assert lib.fdtbx_sf_workspace(0, 10) == 0
    assert lib.fdtbx_structure_factors(ctypes.byref(cell), 10, *([None] * 7), 1, None, 10, None, None, None, 0, None) == -1


def test_model_checks(lib):
    import workloads as W
    from paper_2608_23245_amd import binding as B
    wl = W.config0()
    m = B.make_model(wl)
    assert lib.fdtbx_pattern_workspace(ctypes.byref(m), 150, 1000) > 0
    for field, val in [("sigma_theta", 0.0)]:
        m2 = B.make_model(wl)
        setattr(m2.dis, field, val)
        m2.dis.gamma_theta = 0.0
        assert lib.fdtbx_pattern_workspace(ctypes.byref(m2), 150, 1000) == 0
    m3 = B.make_model(wl)
    m3.geom.distance = -1.0
    assert lib.fdtbx_pattern_workspace(ctypes.byref(m3), 150, 1000) == 0
    m4 = B.make_model(wl)
    m4.quad.n_nodes = 0
    assert lib.fdtbx_pattern_workspace(ctypes.byref(m4), 150, 1000) == 0
    m5 = B.make_model(wl)
    m5.dis.g[0] = float("nan")
    assert lib.fdtbx_pattern_workspace(ctypes.byref(m5), 150, 1000) == 0
    for tilt, ok in ((0.3, True), (-1.5, True), (1.6, False), (float("nan"), False)):
        m6 = B.make_model(wl)
        m6.geom.tilt = tilt
        assert (lib.fdtbx_pattern_workspace(ctypes.byref(m6), 150, 1000) > 0) == ok, tilt
    assert lib.fdtbx_pixel_map(ctypes.byref(m6.geom), ctypes.c_void_p(8), ctypes.c_void_p(8), None) == -2
    # pattern call with a workspace that is too small is rejected before any launch
    rc = lib.fdtbx_profile_pattern(ctypes.byref(m), ctypes.c_void_p(8), 150, ctypes.c_void_p(8), ctypes.c_void_p(8), 1000,
                                   None, ctypes.c_void_p(8), 16, None)
    assert rc == -3


def test_empty_inputs_are_valid_calls(lib):
    """n_hkl = 0 (an empty shell) and n_atoms = 0 are valid: the calls below return before
    any device work, with NULL per-reflection (or per-atom) pointers."""
    import workloads as W
    from paper_2608_23245_amd import binding as B
    m = B.make_model(W.config0())
    cell = m.cell
    assert lib.fdtbx_pattern_workspace(ctypes.byref(m), 0, 1000) > 0
    assert lib.fdtbx_pattern_workspace(ctypes.byref(m), -1, 1000) == 0
    assert lib.fdtbx_backward_workspace(0, 10) > 0
    assert lib.fdtbx_reflection_prep(ctypes.byref(m), None, 0, None, None, None, None) == 0
    assert lib.fdtbx_reflection_prep(ctypes.byref(m), None, -1, None, None, None, None) == -1
    assert lib.fdtbx_cyl_records(ctypes.byref(m), None, 0, None, None) == 0
    assert lib.fdtbx_structure_factors(ctypes.byref(cell), 10, *([None] * 7), 1, None, 0, None, None, None, 0, None) == 0
    assert lib.fdtbx_profile_adjoint(ctypes.byref(m), *([None] * 7), 0, None, None, None) == 0
    assert lib.fdtbx_sf_adjoint(ctypes.byref(cell), 0, *([None] * 7), 1, None, 5, *([None] * 7), None, 0, None) == 0
    assert lib.fdtbx_structure_factors(ctypes.byref(cell), -1, *([None] * 7), 1, None, 5, None, None, None, 0, None) == -1


def test_batch_entries_check_and_setup_envelope(lib):
    """fdtbx_batch_entry_init records the set-up g and N_base (the culling lists' envelope) and
    clears the stale word; fdtbx_batch_entries_check rejects a scattering-factor row count
    outside 1..16 (the batched kernels' LDS tables hold 16 rows) and negative offsets, on the
    host, before any upload."""
    import workloads as W
    from paper_2608_23245_amd import binding as B
    wl = W.config1()
    m = B.make_model(wl)
    ents = (B.BatchEntry * 2)()
    for e in ents:
        assert lib.fdtbx_batch_entry_init(ctypes.byref(m), ctypes.byref(e)) == 0
        e.n_types = 4
    assert list(ents[0].setup_g) == list(wl.dis.g) and list(ents[0].setup_N_base) == list(wl.dis.N_base)
    assert ents[0].stale == 0
    assert lib.fdtbx_batch_entries_check(ctypes.byref(ents), 2) == 0
    for bad in (0, 17, -3):
        ents[1].n_types = bad
        assert lib.fdtbx_batch_entries_check(ctypes.byref(ents), 2) == -1, bad
        assert "n_types" in lib.fdtbx_error_string(-1).decode()
    ents[1].n_types = 16
    assert lib.fdtbx_batch_entries_check(ctypes.byref(ents), 2) == 0
    ents[1].pair_off = -1
    assert lib.fdtbx_batch_entries_check(ctypes.byref(ents), 2) == -1
    assert lib.fdtbx_batch_entries_check(None, 2) == -1


def test_deterministic_adjoint_host_checks(lib):
    """The fixed-order adjoint's entry points check their sizes on the host: the pair order
    takes fewer than 2^31 pairs, empty inputs are valid, null outputs are refused."""
    import workloads as W
    from paper_2608_23245_amd import binding as B
    m = B.make_model(W.config0())
    assert lib.fdtbx_pair_transpose(10, ctypes.c_void_p(8), 1 << 31, None, ctypes.c_void_p(8), ctypes.c_void_p(8),
                                    ctypes.c_void_p(8), 1 << 40, None) == -5
    assert lib.fdtbx_pair_transpose(-1, None, 0, None, None, None, None, 0, None) == -1
    assert lib.fdtbx_pair_transpose(0, None, 0, None, None, None, None, 0, None) == 0
    assert lib.fdtbx_pair_reduce(0, None, None, None, None, 0, None, None) == 0
    assert lib.fdtbx_pair_reduce(5, None, None, None, None, 0, None, None) == -1
    assert lib.fdtbx_profile_adjoint_pairs(ctypes.byref(m), *([None] * 7), 0, 0, None, None, None) == 0
    assert lib.fdtbx_profile_adjoint_pairs(ctypes.byref(m), *([None] * 7), 10, 100, None, None, None) == -1
    assert lib.fdtbx_backward_deterministic_workspace(-1, 0, 10) == 0
    assert lib.fdtbx_backward_deterministic_workspace(0, 0, 10) > 0


def test_noalloc_backward_host_checks(lib):
    """fdtbx_pattern_backward_noalloc refuses, on the host and before any HIP call, a problem
    whose backward workspace exceeds the library's scratch array, and negative sizes; the
    header's array size is the binding's."""
    from paper_2608_23245_amd import binding as B
    src = open(HEADER).read()
    m = re.search(r"#define FDTBX_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == B.NOALLOC_SCRATCH_BYTES
    n_big = 2_000_000
    assert lib.fdtbx_backward_workspace(n_big, 0) > B.NOALLOC_SCRATCH_BYTES
    assert lib.fdtbx_backward_workspace(1_000_000, 0) <= B.NOALLOC_SCRATCH_BYTES
    args = [None, None, n_big, None, None, None, 0, 0, 0] + [None] * 7 + [1] + [None] * 8
    assert lib.fdtbx_pattern_backward_noalloc(*args) == -3
    assert b"scratch" in lib.fdtbx_error_string(-3)
    with_atoms = list(args)
    with_atoms[2], with_atoms[8], with_atoms[17] = 200_000, 20_000, ctypes.c_void_p(8)  # d_x given: atoms count
    assert lib.fdtbx_backward_workspace(200_000, 0) <= B.NOALLOC_SCRATCH_BYTES
    assert lib.fdtbx_backward_workspace(200_000, 20_000) > B.NOALLOC_SCRATCH_BYTES
    assert lib.fdtbx_pattern_backward_noalloc(*with_atoms) == -3
    neg = list(args)
    neg[2] = -1
    assert lib.fdtbx_pattern_backward_noalloc(*neg) == -1


def test_node_rows(lib):
    """Node table size: n^2 node records plus ceil(n/4)^2 block records; 0 outside 1..256."""
    from paper_2608_23245_amd import binding as B
    assert B.NODE_BLOCK == 4
    for n, rows in ((1, 2), (4, 17), (10, 109), (64, 4096 + 256), (96, 9216 + 576), (256, 65536 + 4096)):
        assert lib.fdtbx_node_rows(n) == rows == B.node_rows(n)
    assert lib.fdtbx_node_rows(0) == 0 and lib.fdtbx_node_rows(257) == 0


def test_struct_layouts_match_binding(lib):
    """The ctypes mirrors of the ABI structs have the library's sizes, and host checks
    reject a lineshape outside the three defined and a non-finite damping."""
    import workloads as W
    from paper_2608_23245_amd import binding as B
    assert lib.fdtbx_batch_entry_size() == ctypes.sizeof(B.BatchEntry)
    assert B.N_GLOBALS == 11 and B.LINESHAPES == W.LINESHAPES
    wl = W.config0()
    for ls, ok in ((0, True), (1, True), (2, True), (3, False), (-1, False)):
        m = B.make_model(wl)
        m.dis.lineshape = ls
        assert (lib.fdtbx_pattern_workspace(ctypes.byref(m), 150, 1000) > 0) == ok, ls
    m = B.make_model(wl)
    m.dis.B_axis[1] = float("inf")
    assert lib.fdtbx_pattern_workspace(ctypes.byref(m), 150, 1000) == 0



def test_tile_grid(lib):
    from paper_2608_23245_amd import binding as B
    g = B.Geometry(1.0, 100.0, 0.1, 37, 23, 18.5, 11.5, 0.0, 0)
    tx, ty = ctypes.c_int32(0), ctypes.c_int32(0)
    for tw, want in [(0, (5, 3)), (2, (19, 1)), (4, (10, 2)), (8, (5, 3)), (16, (3, 6)), (32, (2, 12))]:
        g.tile_w = tw
        assert lib.fdtbx_tile_grid(ctypes.byref(g), ctypes.byref(tx), ctypes.byref(ty)) == 0
        assert (tx.value, ty.value) == want, tw
    for bad in (1, 3, 6, 64, -8):
        g.tile_w = bad
        assert lib.fdtbx_tile_grid(ctypes.byref(g), ctypes.byref(tx), ctypes.byref(ty)) == -1
        assert "tile_w" in lib.fdtbx_error_string(-1).decode()


def test_mirror_fold_conditions(lib):
    from paper_2608_23245_amd import binding as B
    tx, ty = ctypes.c_int32(0), ctypes.c_int32(0)
    ok = B.Geometry(1.0, 100.0, 0.1, 48, 23, 24.0, 11.5, 0.3, 16, 1)
    assert lib.fdtbx_tile_grid(ctypes.byref(ok), ctypes.byref(tx), ctypes.byref(ty)) == 0
    assert (tx.value, ty.value) == (3, 6)      # every tile column is still in the grid
    bad = {
        "left-right fold": [B.Geometry(1.0, 100.0, 0.1, 48, 23, 24.2, 11.5, 0.0, 16, 1),   # beam off the middle
                            B.Geometry(1.0, 100.0, 0.1, 40, 23, 20.0, 11.5, 0.0, 16, 1)],  # width not a multiple of 16
        "up-down fold": [B.Geometry(1.0, 100.0, 0.1, 48, 23, 24.0, 11.5, 0.0, 16, 2),      # height not a multiple of 4
                         B.Geometry(1.0, 100.0, 0.1, 48, 24, 24.0, 12.0, 0.1, 16, 2),      # tilted fibre
                         B.Geometry(1.0, 100.0, 0.1, 48, 24, 24.0, 12.3, 0.0, 16, 3),      # beam off the middle row
                         B.Geometry(1.0, 100.0, 0.1, 48, 24, 24.0, 12.0, 0.0, 16, 2, 0, 0, 0.2)],  # tilted detector
        "mirror must be": [B.Geometry(1.0, 100.0, 0.1, 48, 24, 24.0, 12.0, 0.0, 16, m) for m in (-1, 4)],
    }
    for msg, geoms in bad.items():
        for g in geoms:
            assert lib.fdtbx_tile_grid(ctypes.byref(g), ctypes.byref(tx), ctypes.byref(ty)) == -1
            assert msg in lib.fdtbx_error_string(-1).decode()
    for m in (2, 3):
        g = B.Geometry(1.0, 100.0, 0.1, 48, 24, 24.0, 12.0, 0.0, 16, m)
        assert lib.fdtbx_tile_grid(ctypes.byref(g), ctypes.byref(tx), ctypes.byref(ty)) == 0
        assert (tx.value, ty.value) == (3, 6)
    # the launch order covers the left 3 of the 6 tile columns of 8 pixels (3 x 3 tiles, padded
    # to whole rounds of the 8 XCDs), against 6 x 3 without the fold; with the up-down fold too
    # (24 rows of 8-row tiles), the top 2 of the 3 tile rows
    g = B.Geometry(1.0, 100.0, 0.1, 48, 23, 24.0, 11.5, 0.0, 8, 1)
    lib.fdtbx_tile_order_size.restype = ctypes.c_int64
    assert lib.fdtbx_tile_order_size(ctypes.byref(g)) == 16
    g.mirror = 0
    assert lib.fdtbx_tile_order_size(ctypes.byref(g)) == 24
    g = B.Geometry(1.0, 100.0, 0.1, 48, 24, 24.0, 12.0, 0.0, 8, 3)
    assert lib.fdtbx_tile_order_size(ctypes.byref(g)) == 8
    g.mirror = 2
    assert lib.fdtbx_tile_order_size(ctypes.byref(g)) == 16


def test_tile_waves_values(lib):
    from paper_2608_23245_amd import binding as B
    tx, ty = ctypes.c_int32(0), ctypes.c_int32(0)
    g = B.Geometry(1.0, 100.0, 0.1, 48, 23, 20.0, 11.5, 0.0, 8, 0, 0)
    for w in (0, 1, 2, 4):
        g.tile_waves = w
        assert lib.fdtbx_tile_grid(ctypes.byref(g), ctypes.byref(tx), ctypes.byref(ty)) == 0
    for w in (3, 8, -1):
        g.tile_waves = w
        assert lib.fdtbx_tile_grid(ctypes.byref(g), ctypes.byref(tx), ctypes.byref(ty)) == -1
        assert "tile_waves" in lib.fdtbx_error_string(-1).decode()


def test_launch_waves_explicit(lib):
    """An explicit tile_waves is returned as it is (no device query)."""
    from paper_2608_23245_amd import binding as B
    w = ctypes.c_int32(0)
    for tw in (1, 2, 4):
        g = B.Geometry(1.0, 100.0, 0.1, 48, 23, 24.0, 11.5, 0.0, 8, 1, tw)
        assert lib.fdtbx_launch_waves(ctypes.byref(g), ctypes.byref(w)) == 0 and w.value == tw
    assert lib.fdtbx_launch_waves(None, ctypes.byref(w)) == -1


def test_detector_tilt_checks(lib):
    """The detector tilt: |det_tilt| < pi/2, and every pixel row in front of the sample."""
    from paper_2608_23245_amd import binding as B
    tx, ty = ctypes.c_int32(0), ctypes.c_int32(0)
    ok = B.Geometry(1.0, 100.0, 0.1, 48, 24, 24.0, 12.0, 0.0, 16, 1, 0, 0, 0.4)
    assert lib.fdtbx_tile_grid(ctypes.byref(ok), ctypes.byref(tx), ctypes.byref(ty)) == 0   # left-right fold kept
    for d in (math.pi / 2, -2.0, float("nan")):
        g = B.Geometry(1.0, 100.0, 0.1, 48, 24, 24.0, 12.0, 0.0, 16, 0, 0, 0, d)
        assert lib.fdtbx_tile_grid(ctypes.byref(g), ctypes.byref(tx), ctypes.byref(ty)) == -2
        assert "detector tilt" in lib.fdtbx_error_string(-2).decode()
    # a row 1000 pixels (100 mm) above the beam on a detector leaning 1.2 rad toward the sample
    behind = B.Geometry(1.0, 100.0, 0.1, 48, 2200, 24.0, 100.0, 0.0, 16, 0, 0, 0, 1.2)
    assert lib.fdtbx_tile_grid(ctypes.byref(behind), ctypes.byref(tx), ctypes.byref(ty)) == -2
    assert "behind the sample" in lib.fdtbx_error_string(-2).decode()
