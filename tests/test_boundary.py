"""The C-ABI library: it loads, exports every declared symbol, and rejects
invalid descriptions before touching the device (no GPU needed)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "gemfdtd.h")


def _declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fdtd_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2405_00814_amd import _lib
    L = _lib.load()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTED)
    assert L.fdtd_version().startswith(b"gemfdtd")


def test_product_path_has_no_cpu_fallback(tmp_path):
    from paper_2405_00814_amd import _lib
    with pytest.raises(RuntimeError):
        _lib.open_library(str(tmp_path / "missing.so"))


def _create(**over):
    from paper_2405_00814_amd import _lib
    from paper_2405_00814_amd.sim import make_desc
    shape = over.pop("shape", (16, 12))
    h = 1e-3
    dt = over.pop("dt", 0.9 / math.sqrt(2) * h / 299792458.0)
    kw = dict(eps_r=None, mu_r=None, sigma=None, npml=None, cpml=None)
    kw.update(over)
    d, keep = make_desc(shape, (h,) * len(shape), dt, stream=0, allocator=False, **kw)
    out = C.c_void_p()
    rc = _lib.load().fdtd_create(C.byref(d), C.byref(out))
    msg = _lib.load().fdtd_last_error().decode()
    return rc, out, msg


@pytest.mark.parametrize("over,code", [
    (dict(shape=(2, 12)), -1),
    (dict(dt=1.0 / (299792458.0 * math.sqrt(2 / 1e-6)) * 1.001), -2),
    (dict(eps_r=np.full((16, 12), 0.5)), -1),
    (dict(eps_r=np.where(np.arange(192).reshape(16, 12) == 7, np.nan, 1.0)), -1),
    (dict(sigma=np.full((16, 12), -1.0)), -1),
    (dict(mu_r=np.full((16, 12), 0.9)), -1),
    (dict(npml=(8, 8, 0, 0)), -1),
    (dict(cpml=dict(kappa_max=0.5)), -1),
])
def test_create_rejects_invalid(over, code):
    rc, out, msg = _create(**over)
    assert rc == code, msg
    assert not out.value
    assert msg


def test_courant_limit_boundary():
    # exactly at the limit is accepted by validation (then needs a device);
    # just above is FDTD_EUNSTABLE
    lim = 1.0 / (299792458.0 * math.sqrt(2 / 1e-6))
    rc, _, _ = _create(dt=lim * (1 + 1e-9))
    assert rc == -2
    rc3, _, _ = _create(shape=(8, 8, 8), dt=1.0 / (299792458.0 * math.sqrt(3 / 1e-6)) * 1.01)
    assert rc3 == -2


def test_null_arguments():
    from paper_2405_00814_amd import _lib
    L = _lib.load()
    assert L.fdtd_create(None, None) == -1
    assert L.fdtd_destroy(None) == 0
    assert L.fdtd_step(None, 1) == -1
    assert L.fdtd_probe(None, None, 0, None) == -1


@pytest.mark.parametrize("n,npml,split", [(19000, 16, 0), (15000, 16, 1)])
def test_graph_size_guard(n, npml, split):
    """The explicit graph's row pointers and columns are int32: a grid whose
    largest layer would hold 2^31 or more nonzeros (19000^2 cells: about 6
    per cell in the H layer; split-field 15000^2: about 10) is refused with
    FDTD_EINVAL before any device work or host-side graph construction,
    although its node count fits."""
    from paper_2405_00814_amd import _lib
    from paper_2405_00814_amd.sim import make_desc
    h = 1e-3
    dt = 0.9 / math.sqrt(2) * h / 299792458.0
    cells = n * n
    assert (4 if split else 3) * cells < 2 ** 31  # nodes fit
    d, keep = make_desc((n, n), (h, h), dt, npml=(npml,) * 4, cpml=dict(split=split), stream=0,
                        allocator=False)
    out = C.c_void_p()
    L = _lib.load()
    rc = L.fdtd_create_graph(C.byref(d), C.byref(out))
    assert rc == -1 and not out.value
    assert b"nonzeros" in L.fdtd_last_error()


def test_stream_copy_argument_rules():
    """fdtd_stream_copy checks its arguments before any device work: NULL
    pointers, a byte count or an address that is not a multiple of 16 give
    FDTD_EINVAL; a zero-byte copy of aligned addresses is a no-op."""
    from paper_2405_00814_amd import _lib
    L = _lib.load()
    v = C.c_void_p
    assert L.fdtd_stream_copy(None, v(0x1000), 16, None) == -1
    assert L.fdtd_stream_copy(v(0x1000), None, 16, None) == -1
    assert L.fdtd_stream_copy(v(0x1000), v(0x2000), 20, None) == -1
    assert L.fdtd_stream_copy(v(0x1004), v(0x2000), 16, None) == -1
    assert L.fdtd_stream_copy(v(0x1000), v(0x2008), 16, None) == -1
    assert b"multiples of 16" in L.fdtd_last_error()
    assert L.fdtd_stream_copy(v(0x1000), v(0x2000), 0, None) == 0


def test_noalloc_probe_rejects_null():
    from paper_2405_00814_amd import _lib
    L = _lib.load()
    assert L.fdtd_probe_noalloc(None, None, 0, None) == -1
