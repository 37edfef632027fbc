"""The C-ABI library loads without a GPU, exports every declared entry point,
passes its host self-test and validates parameters (no device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1701_03637_amd import lbsc
    return lbsc.load_library()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lbsc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbsc_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1701_03637_amd import lbsc
    assert sorted(lbsc.SYMBOLS) == declared_functions()


def test_host_selftest(lib):
    assert lib.lbsc_selftest() == 0


def test_create_validates_and_sizes(lib):
    from paper_1701_03637_amd import lbsc
    h = ctypes.c_void_p()
    p = lbsc.make_params(64, 48, 40, precision="fp32s", sink="faces")
    assert lib.lbsc_create(1, ctypes.byref(p), ctypes.byref(h)) == 0
    pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.lbsc_required_bytes(h, ctypes.byref(pb), ctypes.byref(sb)) == 0
    assert pb.value == 40 * 38 * ((64 * 48 + 63) // 64 * 64) * 4
    nit = ctypes.c_int32()
    assert lib.lbsc_num_items(h, ctypes.byref(nit)) == 0 and nit.value > 0
    # calls that need device buffers report an unbound context
    assert lib.lbsc_step(h, 1) == -2
    assert b"lbsc_bind" in lib.lbsc_last_error(h)
    assert lib.lbsc_destroy(h) == 0
    for bad in (dict(nx=0), dict(tau=(0.5, 1.0)), dict(precision=7), dict(sink=9), dict(phi_delta=(0.1, 0.1))):
        q = lbsc.make_params(8, 8, 8)
        for k, v in bad.items():
            if k == "tau":
                q.tau[0], q.tau[1] = v
            elif k == "phi_delta":
                q.phi_delta[0], q.phi_delta[1] = v
            else:
                setattr(q, k, v)
        assert lib.lbsc_create(1, ctypes.byref(q), ctypes.byref(h)) == -1, bad
    for bad in (dict(plane_pad=-2), dict(plane_pad=(1 << 20) + 1)):
        q = lbsc.make_params(8, 8, 8, **bad)
        assert lib.lbsc_create(1, ctypes.byref(q), ctypes.byref(h)) == -1, bad
    # mixed precisions in one context are rejected
    two = (lbsc.Params * 2)(lbsc.make_params(8, 8, 8, precision="fp32s"), lbsc.make_params(8, 8, 8))
    assert lib.lbsc_create(2, two, ctypes.byref(h)) == -1
    assert lib.lbsc_status_string(-4) == b"non-finite density"


def test_tile_schedule_errors(lib):
    from paper_1701_03637_amd import lbsc
    h = ctypes.c_void_p()
    p = lbsc.make_params(32, 32, 32)
    assert lib.lbsc_create(1, ctypes.byref(p), ctypes.byref(h)) == 0
    for t in (lbsc.Tiles(128, 0, 0, 0, 0), lbsc.Tiles(32, 16, 2, 0, 0), lbsc.Tiles(256, 600, 0, 0, 0), lbsc.Tiles(512, 0, 0, 0, 3)):
        assert lib.lbsc_set_tiles(h, ctypes.byref(t)) == -1
    assert lib.lbsc_set_tiles(h, ctypes.byref(lbsc.Tiles(512, 32, 16, 4, 2))) == 0
    nit = ctypes.c_int32()
    lib.lbsc_num_items(h, ctypes.byref(nit))
    assert nit.value == 1 * 2 * 8
    assert lib.lbsc_set_graph(h, 3) == -1 and lib.lbsc_set_graph(h, 4) == 0
    lib.lbsc_destroy(h)


def test_kernel_variant_resolution(lib):
    """Variant 0 resolves to the pipelined step where every tile's halo has a
    thread per node (and, for FP16N, the rest footprint fits) and the storage
    is FP32S / FP16S / FP16N, or FP64 in 256-thread blocks, else to the
    register-keeping step; an explicit variant 3 that does not fit fails."""
    from paper_1701_03637_amd import lbsc

    def resolve(prec, n, tiles):
        h = ctypes.c_void_p()
        p = lbsc.make_params(*n, precision=prec)
        assert lib.lbsc_create(1, ctypes.byref(p), ctypes.byref(h)) == 0
        rc = lib.lbsc_set_tiles(h, ctypes.byref(lbsc.Tiles(*tiles)))
        out = lbsc.Tiles()
        assert lib.lbsc_get_tiles(h, ctypes.byref(out)) == 0
        lib.lbsc_destroy(h)
        return rc, out.nt, out.variant

    assert resolve("fp32s", (128, 128, 128), (0, 0, 0, 0, 0)) == (0, 512, 3)
    assert resolve("fp16s", (128, 128, 128), (0, 0, 0, 0, 0)) == (0, 512, 3)
    assert resolve("fp64", (128, 128, 128), (0, 0, 0, 0, 0)) == (0, 256, 3)
    assert resolve("fp64", (128, 128, 128), (512, 0, 0, 0, 0)) == (0, 512, 1)
    assert resolve("fp64", (128, 128, 128), (512, 0, 0, 0, 3))[0] == -1
    assert resolve("fp16n", (128, 128, 128), (0, 0, 0, 0, 0)) == (0, 512, 3)
    # 128 x 2 tiles of a 256-wide lattice: 2 (128 + 2) + 2 x 2 = 264 halo nodes
    assert resolve("fp32s", (256, 64, 32), (256, 128, 2, 0, 0)) == (0, 256, 1)
    rc, _, _ = resolve("fp32s", (256, 64, 32), (256, 128, 2, 0, 3))
    assert rc == -1
    assert resolve("fp32s", (256, 64, 32), (512, 128, 4, 0, 3)) == (0, 512, 3)
    assert resolve("fp16n", (64, 64, 64), (256, 64, 4, 0, 3)) == (0, 256, 3)
    assert resolve("fp16n", (256, 64, 32), (256, 128, 2, 0, 3))[0] == -1
    assert resolve("fp16nf", (128, 128, 128), (0, 0, 0, 0, 0)) == (0, 512, 3)
    assert resolve("fp16nf", (256, 64, 32), (256, 128, 2, 0, 3))[0] == -1



def test_default_tiles_split_evenly(lib):
    """Automatic schedules split x, y and z into near-equal parts, with tiles
    of at least 3 rows for the pipelined step and 8 for the register-keeping
    one: a 156^3 box gets full-width tiles of 3 rows (52 tiles; 156 = 3 x 52)
    in 9 chunks, a 300-wide box three 100-wide tiles of 5 rows. Where a row
    is a whole number of 128-byte lines, part boundaries fall on lines: a
    512-wide FP64 box gets eight 64 x 4 tiles rather than seven 73 or 74
    wide, FP32S 128 x 4 tiles, and the pipelined FP16 forms (bound by
    instruction issue, so halo nodes cost more than halo columns) 64-wide
    tiles.
    The 128^3 droplet gets 32 tiles of 128 x 4 in 8 chunks of 16 planes (FP64, 256
    threads: 64 tiles of 64 x 4 in 4 chunks). Chunks shorter than 16 planes
    are made only until the blocks number the 256 CUs: 11 chunks of the
    32-plane box's 24 tiles, one-plane chunks of the 4x4x128 film."""
    from paper_1701_03637_amd import lbsc

    def items(n, prec, tiles=None):
        h = ctypes.c_void_p()
        p = lbsc.make_params(*n, precision=prec)
        assert lib.lbsc_create(1, ctypes.byref(p), ctypes.byref(h)) == 0
        if tiles is not None:
            assert lib.lbsc_set_tiles(h, ctypes.byref(lbsc.Tiles(*tiles))) == 0
        v = ctypes.c_int32()
        assert lib.lbsc_num_items(h, ctypes.byref(v)) == 0
        lib.lbsc_destroy(h)
        return v.value

    assert items((156, 156, 156), "fp32s") == 52 * 9
    assert items((300, 40, 32), "fp32s") == 3 * 8 * 11                  # ceil(256 / 24) chunks
    assert items((384, 40, 32), "fp32s") == 3 * 10 * 9                  # 128 x 4 tiles; ceil(256 / 30) chunks
    assert items((512, 16, 16), "fp64") == 8 * 4 * 8                    # 64 x 4 tiles, not 7 parts of 73
    assert items((512, 20, 16), "fp32s") == 4 * 5 * 13                  # 128 x 4 tiles
    assert items((512, 20, 16), "fp16n") == 8 * 3 * 11                  # 64 x 7: halo columns weigh less
    assert items((128, 128, 128), "fp32s") == 32 * 8
    assert items((128, 128, 128), "fp64") == 64 * 4
    assert items((4, 4, 128), "fp64") == 128
    assert items((4, 4, 128), "fp32s") == 128
    assert items((4, 4, 128), "fp64", (256, 0, 0, 16, 3)) == 8         # explicit chunk length
    # cases where full-width tiles would be too thin (one-plane chunks)
    assert items((200, 9, 16), "fp32s") == 2 * 2 * 16   # 100 x 5 (full width: 2 rows, 5 tiles)
    assert items((100, 9, 16), "fp64") == 2 * 2 * 16    # 50 x 5 (full width: 2 rows, 5 tiles)
    # the keep step asks for 8 rows
    assert items((100, 11, 16), "fp16n", (512, 0, 0, 0, 1)) == 2 * 2 * 16   # 50 x 10 (full width: 5 rows, 3 tiles)
    assert items((100, 11, 16), "fp16n") == 3 * 16                           # pipelined: full width, 5 rows


def test_bench_refuses_more_than_one_gpu():
    """bench.py steps one GPU: --gpus above 1 exits with status 2 and says
    so, before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "--gpus must be 1" in r.stderr


def test_fp16s_with_a_sink_needs_the_flag(lib):
    """Constant-shift FP16 storage with an evaporation sink is refused
    (LBSC_E_UNSUPPORTED) unless LBSC_FLAG_FP16S_SINK is set; FP16S without a
    sink and FP16N with one are accepted."""
    from paper_1701_03637_amd import lbsc
    h = ctypes.c_void_p()
    for sink in ("zmax", "faces", "sphere"):
        p = lbsc.make_params(16, 16, 16, precision="fp16s", sink=sink, sink_radius=6.0)
        assert lib.lbsc_create(1, ctypes.byref(p), ctypes.byref(h)) == -5, sink
        p = lbsc.make_params(16, 16, 16, precision="fp16s", sink=sink, sink_radius=6.0, flags=lbsc.FLAG_FP16S_SINK)
        assert lib.lbsc_create(1, ctypes.byref(p), ctypes.byref(h)) == 0
        assert lib.lbsc_destroy(h) == 0
    for prec, sink in (("fp16s", "none"), ("fp16n", "faces"), ("fp16nf", "faces")):
        p = lbsc.make_params(16, 16, 16, precision=prec, sink=sink)
        assert lib.lbsc_create(1, ctypes.byref(p), ctypes.byref(h)) == 0
        assert lib.lbsc_destroy(h) == 0


def test_wall_and_flag_validation(lib):
    from paper_1701_03637_amd import lbsc
    h = ctypes.c_void_p()
    for kw in (dict(solid_z=2, wall_z=True), dict(solid_z=8), dict(solid_z=-1), dict(flags=2),
               dict(wall_rho=(float("nan"), 0.0))):
        p = lbsc.make_params(8, 8, 8, **kw)
        assert lib.lbsc_create(1, ctypes.byref(p), ctypes.byref(h)) == -1, kw


def test_single_component_validation(lib):
    """The single-component form stores FP64 or FP32S; every instance of a
    context has the same number of components; its step has one variant."""
    from paper_1701_03637_amd import lbsc
    h = ctypes.c_void_p()
    for prec, want in (("fp64", 0), ("fp32s", 0), ("fp16n", -5), ("fp16nf", -5), ("fp16s", -5)):
        p = lbsc.make_params(16, 16, 16, precision=prec, ncomp=1, g=-5.0, psi="exp")
        assert lib.lbsc_create(1, ctypes.byref(p), ctypes.byref(h)) == want, prec
        if want == 0:
            pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
            assert lib.lbsc_required_bytes(h, ctypes.byref(pb), ctypes.byref(sb)) == 0
            elem = 8 if prec == "fp64" else 4
            assert pb.value == 16 * 19 * ((16 * 16 + 63) // 64 * 64) * elem
            assert lib.lbsc_set_tiles(h, ctypes.byref(lbsc.Tiles(256, 0, 0, 0, 3))) == -1
            assert lib.lbsc_set_tiles(h, ctypes.byref(lbsc.Tiles(256, 0, 0, 0, 1))) == 0
            assert lib.lbsc_destroy(h) == 0
    p = lbsc.make_params(8, 8, 8, ncomp=3)
    assert lib.lbsc_create(1, ctypes.byref(p), ctypes.byref(h)) == -1
    two = (lbsc.Params * 2)(lbsc.make_params(8, 8, 8, ncomp=1), lbsc.make_params(8, 8, 8))
    assert lib.lbsc_create(2, two, ctypes.byref(h)) == -1


def test_per_instance_tiles_and_tune_cache_file(lib, tmp_path):
    """Per-instance tile overrides change only their instance's work items;
    the tuning cache file keeps entries of the loaded library's kernel sources and
    skips others."""
    from paper_1701_03637_amd import lbsc
    h = ctypes.c_void_p()
    two = (lbsc.Params * 2)(lbsc.make_params(40, 40, 40, precision="fp32s"),
                            lbsc.make_params(150, 150, 20, precision="fp32s"))
    assert lib.lbsc_create(2, two, ctypes.byref(h)) == 0
    n0 = ctypes.c_int32()
    lib.lbsc_num_items(h, ctypes.byref(n0))
    assert lib.lbsc_set_inst_tiles(h, 0, ctypes.byref(lbsc.Tiles(0, 16, 4, 2, 0))) == 0
    n1 = ctypes.c_int32()
    lib.lbsc_num_items(h, ctypes.byref(n1))
    assert n1.value > n0.value
    t = lbsc.Tiles()
    assert lib.lbsc_get_inst_tiles(h, 0, ctypes.byref(t)) == 0 and (t.tw, t.th, t.nzc) == (16, 4, 2)
    assert lib.lbsc_get_inst_tiles(h, 1, ctypes.byref(t)) == 0 and (t.tw, t.th, t.nzc) == (0, 0, 0)
    assert lib.lbsc_set_inst_tiles(h, 1, ctypes.byref(lbsc.Tiles(0, 600, 0, 0, 0))) == -1
    assert lib.lbsc_set_inst_tiles(h, 2, ctypes.byref(lbsc.Tiles(0, 16, 0, 0, 0))) == -1
    assert lib.lbsc_destroy(h) == 0
    lib.lbsc_tune_cache_clear()
    path = str(tmp_path / "tune.txt")
    kh = lib.lbsc_kernel_hash().decode()
    with open(path, "w") as fh:
        fh.write(f"lbsc-tune 1 {kh} gfx950 64 64 64 1 2 0 0 512 32 0 8 3\n")
        fh.write("lbsc-tune 1 0000000000000000 gfx950 64 64 64 1 2 0 0 256 0 0 0 1\n")
    n = ctypes.c_int32()
    assert lib.lbsc_tune_cache_load(path.encode(), ctypes.byref(n)) == 0 and n.value == 1
    out = str(tmp_path / "out.txt")
    assert lib.lbsc_tune_cache_save(out.encode()) == 0
    lines = open(out).read().split("\n")
    assert lines[0] == f"lbsc-tune 1 {kh} gfx950 64 64 64 1 2 0 0 512 32 0 8 3" and lines[1] == ""
    lib.lbsc_tune_cache_clear()


def test_automatic_plane_skew(lib):
    """plane_pad = -1 (the binding's default) adds 320 elements between
    population planes whose byte stride is a multiple of 64 KiB on planes of
    at least 2^14 nodes, and nothing otherwise; explicit pads round up to 64."""
    from paper_1701_03637_amd import lbsc

    def pop_bytes(nx, ny, nz, precision, pad=-1, ncomp=2):
        h = ctypes.c_void_p()
        p = lbsc.make_params(nx, ny, nz, precision=precision, plane_pad=pad, ncomp=ncomp)
        assert lib.lbsc_create(1, ctypes.byref(p), ctypes.byref(h)) == 0
        pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
        assert lib.lbsc_required_bytes(h, ctypes.byref(pb), ctypes.byref(sb)) == 0
        lib.lbsc_destroy(h)
        return pb.value
    # FP32S: 19 planes of (A, B) pairs of 4-byte elements per slab
    assert pop_bytes(128, 128, 4, "fp32s") == 4 * 38 * (128 * 128 + 320) * 4
    assert pop_bytes(128, 128, 4, "fp32s", pad=0) == 4 * 38 * 128 * 128 * 4
    assert pop_bytes(128, 128, 4, "fp32s", pad=100) == 4 * 38 * (128 * 128 + 128) * 4
    assert pop_bytes(100, 100, 4, "fp32s") == 4 * 38 * ((100 * 100 + 63) // 64 * 64) * 4   # 40 000 B planes
    assert pop_bytes(64, 64, 4, "fp32s") == 4 * 38 * 64 * 64 * 4                             # 2^12 nodes
    # 192 x 128 planes: 192 KiB per FP32S pair plane (skewed), 96 KiB per FP16S one (not)
    assert pop_bytes(192, 128, 2, "fp32s") == 2 * 38 * (192 * 128 + 320) * 4
    assert pop_bytes(192, 128, 2, "fp16s") == 2 * 38 * 192 * 128 * 2
    # FP64 pair planes (16 B per node), FP16N (40 half-elements per node)
    assert pop_bytes(128, 128, 2, "fp64") == 2 * 38 * (128 * 128 + 320) * 8
    assert pop_bytes(128, 128, 2, "fp16n") == 2 * 40 * (128 * 128 + 320) * 2
    assert pop_bytes(128, 128, 2, "fp16nf") == 2 * 40 * (128 * 128 + 320) * 2
    # one component: 19 planes (the buffer ends on a 256-element boundary)
    assert pop_bytes(128, 128, 2, "fp32s", ncomp=1) == -(-2 * 19 * (128 * 128 + 320) // 256) * 256 * 4

