"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol include/lbib.h declares, sizes its buffers, and rejects invalid
arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_1903_03356_amd import lbib

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "lbib.h")


@pytest.fixture(scope="module")
def L():
    return lbib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbib_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert sorted(lbib.EXPORTS) == names


def test_required_bytes(L):
    g = lbib.make_grid(100, 37, 4, 3, 300, 128)
    nxp = 128  # 100 rounded up to whole 64-cell segments
    assert lbib.required_bytes(g, 0) == -(-9 * nxp * 37 * 4 // 256) * 256
    assert lbib.required_bytes(g, 1) == lbib.required_bytes(g, 0)
    assert lbib.required_bytes(g, 2) >= 2 * nxp * 37 * 16
    assert lbib.required_bytes(g, 3) >= 2 * 37 * 2 * 4
    assert lbib.required_bytes(g, 7) >= 3 * 100 * 37 * 8
    assert lbib.required_bytes(g, 8) == 0  # unknown buffer id
    g8 = lbib.make_grid(100, 37, 8, 3, 300, 128)
    assert lbib.required_bytes(g8, 0) == 2 * lbib.required_bytes(g, 0)
    for i in range(8):
        assert lbib.required_bytes(g, i) % 256 == 0
    # a row of 1024 cells is padded by one segment (no power-of-two strides)
    g2 = lbib.make_grid(1024, 16, 4)
    assert lbib.required_bytes(g2, 0) == -(-9 * 1088 * 16 * 4 // 256) * 256
    bad = lbib.make_grid(4, 37, 4)
    assert all(lbib.required_bytes(bad, i) == 0 for i in range(8))
    bad = lbib.make_grid(100, 37, 2)
    assert lbib.required_bytes(bad, 0) == 0


def _create(L, grid, tau, walls, nbuf=lbib.NUM_BUFFERS, null=False):
    ptrs = (C.c_void_p * lbib.NUM_BUFFERS)(*([None] * lbib.NUM_BUFFERS if null else
                                            [C.c_void_p(256 * (i + 1)) for i in range(lbib.NUM_BUFFERS)]))
    h = C.c_void_p()
    rc = L.lbib_create(C.byref(grid), tau, C.byref(walls), ptrs, nbuf, None, C.byref(h))
    return rc, h


def test_create_rejects_invalid_arguments(L):
    g = lbib.make_grid(64, 64, 8, 1, 64, 64)
    w = lbib.lbib_walls(1, 0, 0.0, 0.0, 0.0, 0, 0.0, 0.0)
    rc, h = _create(L, g, 0.5, w)
    assert rc == lbib.EINVAL and not h.value
    assert b"tau" in L.lbib_last_error(None)
    rc, _ = _create(L, g, float("nan"), w)
    assert rc == lbib.EINVAL
    rc, _ = _create(L, lbib.make_grid(7, 64, 8), 0.8, w)
    assert rc == lbib.EINVAL
    rc, _ = _create(L, lbib.make_grid(64, 64, 2), 0.8, w)
    assert rc == lbib.EINVAL
    rc, _ = _create(L, lbib.make_grid(64, 64, 4, 1, 64, 5000), 0.8, w)
    assert rc == lbib.ECAPACITY
    w2 = lbib.lbib_walls(2, 0, 0.0, 0.0, 0.0, 0, 0.0, 0.0)
    rc, _ = _create(L, g, 0.8, w2)
    assert rc == lbib.EINVAL and b"periodic_x" in L.lbib_last_error(None)
    # open channel: outlet density, stationary walls, no body force, no periodic y
    for args in ((0, 0, 0.0, 0.0, 0.0, 0, 0.0, 0.0, 0.01, 0.0),
                 (0, 0, 0.0, 0.01, 0.0, 0, 0.0, 0.0, 0.01, 1.0),
                 (0, 0, 0.0, 0.0, 1e-6, 0, 0.0, 0.0, 0.01, 1.0),
                 (0, 1, 0.0, 0.0, 0.0, 0, 0.0, 0.0, 0.01, 1.0),
                 (0, 0, 0.0, 0.0, 0.0, 0, 0.0, 0.0, 0.5, 1.0)):
        rc, _ = _create(L, g, 0.8, lbib.lbib_walls(*args))
        assert rc == lbib.EINVAL, args
    # the inlet parabola as initial state needs an open channel
    rc, _ = _create(L, g, 0.8, lbib.lbib_walls(1, 0, 0.0, 0.0, 0.0, 4, 0.0, 0.0, 0.0, 1.0))
    assert rc == lbib.EINVAL
    wbad = lbib.lbib_walls(1, 0, float("inf"), 0.0, 0.0, 0, 0.0, 0.0)
    rc, _ = _create(L, g, 0.8, wbad)
    assert rc == lbib.EINVAL
    wprof = lbib.lbib_walls(1, 0, 0.0, 0.0, 0.0, 7, 0.0, 0.0)
    rc, _ = _create(L, g, 0.8, wprof)
    assert rc == lbib.EINVAL
    rc, _ = _create(L, g, 0.8, w, nbuf=3)
    assert rc == lbib.EINVAL
    rc, _ = _create(L, g, 0.8, w, null=True)
    assert rc == lbib.EINVAL and b"NULL" in L.lbib_last_error(None)


def test_null_context_calls(L):
    assert L.lbib_step(None, 1, 0) == lbib.EINVAL
    assert L.lbib_check(None, None) == lbib.EINVAL
    assert L.lbib_steps_done(None) == -1
    assert L.lbib_get_state(None, 0, 0, None, 0, 0) == lbib.EINVAL
    assert L.lbib_set_timing(None, 1) == lbib.EINVAL
    assert L.lbib_set_overlap(None, 1) == lbib.EINVAL
    assert L.lbib_set_contact(None, 2.0) == lbib.EINVAL
    assert L.lbib_adjoint_bytes(None, 10, 0) == 0
    assert L.lbib_set_graph(None, 1) == lbib.EINVAL
    assert L.lbib_graph_replays(None) == -1
    assert L.lbib_set_tile(None, 1, 0, 0) == lbib.EINVAL
    assert L.lbib_autotune(None, 5, None, None, None, None, 0) == lbib.EINVAL
    d = C.c_double()
    ks = (C.c_double * 4)()
    assert L.lbib_adjoint(None, 10, 0, 1, 0, 0, None, 0, C.byref(d), C.byref(d), ks, 4) == lbib.EINVAL
    L.lbib_destroy(None)


def test_one_hip_runtime_whatever_the_import_order():
    """Loading the library before torch must not map a second HIP runtime next
    to torch's own (two runtimes share no streams or synchronisation)."""
    import subprocess
    import sys
    code = ("from paper_1903_03356_amd import lbib\n"
            "lbib.load()\n"
            "import torch\n"
            "torch.zeros(1)\n"
            "paths = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(paths))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1", out.stdout


def test_missing_library_fails_loudly():
    """Without the built HIP library the binding raises ImportError: there is
    no CPU fallback for any step of the path."""
    import subprocess
    import sys
    code = ("from paper_1903_03356_amd import lbib\n"
            "lbib.LIB_PATH = '/nonexistent/liblbib.so'\n"
            "try:\n"
            "    lbib.load()\n"
            "except ImportError as e:\n"
            "    print('ImportError', 'build' in str(e))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "ImportError True", out.stdout


def test_noalloc_gradient_declared_with_its_scratch_size(L):
    """The allocation-free gradient call is exported, its static workspace size
    in the header matches the binding's constant, and it rejects a NULL
    context before touching a device."""
    text = open(HEADER).read()
    m = re.search(r"#define\s+LBIB_ADJOINT_SCRATCH_BYTES\s+\((\d+)u \* (\d+)u \* (\d+)u\)", text)
    assert m, "LBIB_ADJOINT_SCRATCH_BYTES not found"
    size = int(m.group(1)) * int(m.group(2)) * int(m.group(3))
    assert size == lbib.ADJOINT_SCRATCH_BYTES == 64 << 20
    J, g = C.c_double(), C.c_double()
    ks = (C.c_double * 4)()
    rc = L.lbib_adjoint_noalloc(None, 10, 0, 1, 0, 0, C.byref(J), C.byref(g), ks, 4)
    assert rc == lbib.EINVAL


def test_membrane_limits_arguments(L):
    """lbib_set_limits rejects a NULL context before touching a device."""
    assert L.lbib_set_limits(None, 1.0, 0.05) == lbib.EINVAL
