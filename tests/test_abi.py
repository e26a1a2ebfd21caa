"""The C-ABI library loads and exports every entry point include/spdhg.h declares, and
host-side argument validation works (no GPU needed: these calls fail before any HIP
call or only do host arithmetic)."""
import ctypes
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spdhg.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1808_07150_amd import build as b
    if not b.up_to_date():
        b.build()
    import paper_1808_07150_amd as P
    return P.load_library()


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spdhg_[a-z0-9_]+)\s*\(", text)))


def test_exports_match_header(lib):
    names = declared_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    import paper_1808_07150_amd.spdhg as S
    assert sorted(S.EXPORTED) == names
    net = declared_functions(os.path.join(ROOT, "include", "spdhg_net.h"))
    assert len(net) >= 12
    for n in net:
        assert hasattr(lib, n), n
    from paper_1808_07150_amd import warmstart
    assert sorted(warmstart.NET_EXPORTED) == net


def test_subset_bins_and_validation(lib):
    import paper_1808_07150_amd as P
    g = synth.mmr()
    assert P.subset_bins(g, 21, 0) == 12 * 837 * 344
    assert P.subset_bins(g, 21, -1) == 252 * 837 * 344
    g2 = synth.Geometry(nx=8, ny=8, nz=1, vx=1, vy=1, vz=1, n_rad=9, d_rad=1, n_ang=10)
    assert P.subset_bins(g2, 4, 0) == 3 * 9 and P.subset_bins(g2, 4, 3) == 2 * 9
    assert P.subset_bins(g2, 4, 4) == -1  # subset out of range
    bad = P.cgeom(g2)
    bad.seg_planes[0] = 2  # nz - N odd
    assert lib.spdhg_subset_bins(ctypes.byref(bad), 1, 0) == -1
    assert b"segment" in lib.spdhg_last_error()


def test_workspace_bytes(lib):
    import paper_1808_07150_amd as P
    g = synth.mmr()
    n = ctypes.c_size_t()
    rc = lib.spdhg_workspace_bytes(ctypes.byref(P.cgeom(g)), ctypes.byref(P.cparams(21, "tv")),
                                   ctypes.byref(n))
    assert rc == 0
    nb, nv = 252 * 837 * 344, 344 * 344 * 127
    # private b, r, mult; y, sigma; x (2), z, T, scratch, prior duals (2 x 3)
    assert 4 * (5 * nb + 11 * nv) < n.value < 4 * (5 * nb + 11 * nv) * 1.1
    rc = lib.spdhg_workspace_bytes(ctypes.byref(P.cgeom(g)), ctypes.byref(P.cparams(300, "tv")),
                                   ctypes.byref(n))
    assert rc == -1  # more subsets than angles
    p = P.cparams(21, "tv")
    p.rho = 1.0
    assert lib.spdhg_workspace_bytes(ctypes.byref(P.cgeom(g)), ctypes.byref(p),
                                     ctypes.byref(n)) == -1


def test_compensated_flag_workspace(lib):
    """The compensated primal step adds the low parts of z and x (8 bytes per voxel);
    it is refused with TGV and unknown flag bits are refused."""
    import paper_1808_07150_amd as P
    g = synth.mmr(nxy=40, n_rad=44, n_ang=24)
    nv = g.nx * g.ny * g.nz
    sizes = []
    for comp in (False, True):
        n = ctypes.c_size_t()
        assert lib.spdhg_workspace_bytes(ctypes.byref(P.cgeom(g)),
                                         ctypes.byref(P.cparams(6, "dtv", compensated=comp)),
                                         ctypes.byref(n)) == 0
        sizes.append(n.value)
    assert sizes[1] - sizes[0] == (8 * nv + 255) // 256 * 256
    n = ctypes.c_size_t()
    assert lib.spdhg_workspace_bytes(ctypes.byref(P.cgeom(g)),
                                     ctypes.byref(P.cparams(6, "tgv", compensated=True)),
                                     ctypes.byref(n)) == -7
    assert b"TGV" in lib.spdhg_last_error()
    p = P.cparams(6, "tv")
    p.flags = 8
    assert lib.spdhg_workspace_bytes(ctypes.byref(P.cgeom(g)), ctypes.byref(p),
                                     ctypes.byref(n)) == -1


def test_null_arguments_rejected(lib):
    import paper_1808_07150_amd as P
    g = P.cgeom(synth.slice64_2d())
    assert lib.spdhg_project(ctypes.byref(g), 10, 0, None, None, None, None, 0, None) == -1
    assert lib.spdhg_backproject(ctypes.byref(g), 10, 0, None, None, None, None, 0,
                                 None) == -1
    assert lib.spdhg_normalised_backprojection(ctypes.byref(g), None, None, None, None, None,
                                               0, None) == -1
    ctx = ctypes.c_void_p()
    assert lib.spdhg_init(ctypes.byref(ctx), ctypes.byref(g),
                          ctypes.byref(P.cparams(10, "tv")), None, None, None, None, None,
                          None, 0, None) == -1
    assert lib.spdhg_iterate(None, 1, None) == -1
    assert lib.spdhg_set_walk(None, 0) == -1
    assert lib.spdhg_set_profiling_kinds(None, 2) == -1


def test_operator_workspace(lib):
    """The stand-alone operator calls take their scratch from the caller: the size query,
    and the NULL / misaligned / too-small workspace errors (raised before any HIP call)."""
    import paper_1808_07150_amd as P
    g = synth.mmr()
    n = P.op_workspace_bytes(g)
    nv, np_, nb = 344 * 344 * 127, 837, 252 * 837 * 344
    # two images, 16 angles of rows and the partials, plus the tables
    assert 4 * (2 * nv + 16 * 344 * np_) + 8 * (nb // 256) <= n
    assert n < 4 * (2 * nv + 16 * 344 * np_) + 8 * (nb // 256) + (4 << 20)
    cg = P.cgeom(synth.slice64_2d())
    fake = ctypes.c_void_p(0x10000)  # never dereferenced: the checks fail first
    for ws, nbytes in ((None, 1 << 20), (ctypes.c_void_p(0x10004), 1 << 30), (fake, 16)):
        rc = lib.spdhg_project(ctypes.byref(cg), 10, 0, None, fake, fake, ws, nbytes, None)
        assert rc == -5, lib.spdhg_last_error()
        rc = lib.spdhg_backproject(ctypes.byref(cg), 10, 0, None, fake, fake, ws, nbytes, None)
        assert rc == -5, lib.spdhg_last_error()
        d = ctypes.c_double()
        rc = lib.spdhg_nnz(ctypes.byref(cg), 10, 0, ctypes.byref(d), ws, nbytes, None)
        assert rc == -5, lib.spdhg_last_error()


def test_library_allocates_no_device_memory():
    """Device memory belongs to the caller: no allocation or free call in the library's
    sources (the workspaces come in as arguments)."""
    csrc = os.path.join(ROOT, "paper_1808_07150_amd", "csrc")
    banned = re.compile(r"\bhip(Malloc|MallocAsync|MallocManaged|ExtMallocWithFlags|Free|"
                        r"FreeAsync|HostMalloc|HostFree|MallocPitch|Malloc3D)\s*\(")
    for name in sorted(os.listdir(csrc)):
        text = open(os.path.join(csrc, name)).read()
        assert not banned.search(text), name


def test_scanner_model_geometry_on_the_host(lib):
    """The library's own count of span-compressed data planes (host code) matches the
    mMR's 837 (and the oracle's count on a small geometry); invalid scanner geometries are
    rejected with a shape error before anything reaches a GPU."""
    import dataclasses

    import paper_1808_07150_amd as P
    from oracle import projector as OP
    g = synth.mmr_scanner()
    assert P.subset_bins(g, 21, 0) == 12 * 837 * 344
    assert P.subset_bins(g, 21, -1) == 252 * 837 * 344
    small = synth.scanner_small()
    assert P.subset_bins(small, 1, -1) == small.n_ang * OP.n_data_planes(small) * small.n_rad
    span1 = dataclasses.replace(small, span=0)
    assert P.subset_bins(span1, 1, -1) == small.n_ang * small.n_planes * small.n_rad
    for bad in (dict(span=4), dict(span=1), dict(det_radius=0.0),
                dict(det_radius=30.0)):  # bin angles past 1.5 rad
        c = P.cgeom(small)
        for k, v in bad.items():
            setattr(c, k, v)
        assert lib.spdhg_subset_bins(ctypes.byref(c), 1, 0) == -1, bad
    # span compression needs the ring-pair segments
    c = P.cgeom(synth.small_3d())
    c.span = 3
    assert lib.spdhg_subset_bins(ctypes.byref(c), 1, 0) == -1
    assert P.op_workspace_bytes(g) > 0
