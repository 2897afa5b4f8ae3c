"""The C ABI library on the CPU: it loads, exports every symbol that
include/*.h declares, and rejects bad arguments before touching a device."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1206_4973_amd", "libfsp.so")


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \t\*]*?\b(fsp_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.fail("libfsp.so is not built (python -m paper_1206_4973_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = _declared()
    for want in ("fsp_load_instance", "fsp_free_instance", "fsp_bound_pool",
                 "fsp_status_string", "fsp_instance_info"):
        assert want in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings(L):
    L.fsp_status_string.restype = ctypes.c_char_p
    for rc, word in ((0, b"ok"), (-1, b"invalid"), (-2, b"memory"), (-3, b"HIP"),
                     (-4, b"unsupported"), (-99, b"unknown")):
        assert word in L.fsp_status_string(rc)


def _load(L, p, n=None, m=None):
    L.fsp_load_instance.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    n = p.shape[0] if n is None else n
    m = p.shape[1] if m is None else m
    ptr = p.ctypes.data_as(ctypes.c_void_p) if p is not None else None
    return L.fsp_load_instance(ptr, n, m, ctypes.byref(h)), h


def test_load_rejects_bad_arguments_without_a_device(L):
    p = np.ones((5, 4), np.int32)
    assert _load(L, p, n=0)[0] == -1
    assert _load(L, p, m=1)[0] == -1
    assert _load(L, np.ones((5, 21), np.int32))[0] == -4         # m above 20
    assert _load(L, np.ones((256, 4), np.int32))[0] == -4        # n above 255
    q = p.copy(); q[2, 1] = -3
    assert _load(L, q)[0] == -1                                   # negative time
    q = p.copy(); q[2, 1] = 40000
    assert _load(L, q)[0] == -4                                   # time above 32767
    q = np.full((3, 4), 20000, np.int32)
    assert _load(L, q)[0] == -4                                   # job total above 65535
    L.fsp_load_instance.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_void_p]
    assert L.fsp_load_instance(p.ctypes.data_as(ctypes.c_void_p), 5, 4, None) == -1
    h = ctypes.c_void_p()
    L.fsp_load_instance.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_void_p)]
    assert L.fsp_load_instance(None, 5, 4, ctypes.byref(h)) == -1


def test_other_entry_points_reject_null(L):
    L.fsp_free_instance.argtypes = [ctypes.c_void_p]
    assert L.fsp_free_instance(None) == 0
    L.fsp_instance_info.argtypes = [ctypes.c_void_p] * 4
    assert L.fsp_instance_info(None, None, None, None) == -1
    L.fsp_instance_path.argtypes = [ctypes.c_void_p] * 2
    assert L.fsp_instance_path(None, None) == -1
    L.fsp_bound_pool.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.c_void_p]
    assert L.fsp_bound_pool(None, 10, None, None) == -1
    L.fsp_bound_pool_one_machine.argtypes = [ctypes.c_void_p, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_void_p]
    assert L.fsp_bound_pool_one_machine(None, 10, None, None) == -1


def test_load_flags_checked_before_device_work(L):
    """fsp_load_instance_ex rejects unknown flag bits with FSP_EINVAL before it
    touches a device (so this runs without a GPU) and leaves *out NULL."""
    L.fsp_load_instance_ex.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]
    p = np.ones((4, 3), np.int32)
    for flags in (4, 8, -1, 1 << 30):
        h = ctypes.c_void_p(1)
        rc = L.fsp_load_instance_ex(p.ctypes.data_as(ctypes.c_void_p), 4, 3, flags,
                                    ctypes.byref(h))
        assert rc == -1 and not h.value


def test_bound_choice_rule(L):
    """The host rule of the per-depth bound choice on hand-made counts:
    deepest first, a depth takes the one-machine bound when it had nodes, the
    next depth keeps the pair bound, and (elim2 - elim1) * (n - d) <=
    total / 2."""
    L.fsp_bound_choice_rule.argtypes = [ctypes.c_int32] + [ctypes.c_void_p] * 4
    L.fsp_bound_choice_rule.restype = ctypes.c_int

    def rule(n, total, e1, e2):
        arrs = [np.zeros(256, np.uint32) for _ in range(3)]
        for a, v in zip(arrs, (total, e1, e2)):
            for d, x in v.items():
                a[d] = x
        mask = np.zeros(8, np.uint32)
        rc = L.fsp_bound_choice_rule(n, *[a.ctypes.data_as(ctypes.c_void_p) for a in arrs],
                                     mask.ctypes.data_as(ctypes.c_void_p))
        assert rc == 0
        return [32 * w + b for w in range(8) for b in range(32) if (int(mask[w]) >> b) & 1]

    n = 10
    flat = {d: 1000 for d in range(1, n)}
    # nothing only the pair bound eliminates: every other depth from n - 1 up
    assert rule(n, flat, {}, {}) == [1, 3, 5, 7, 9]
    # depth 9 (one child per survivor): 500 extra of 1000 is exactly half
    assert rule(n, flat, {}, {9: 500}) == [1, 3, 5, 7, 9]
    assert rule(n, flat, {}, {9: 501}) == [2, 4, 6, 8]
    # depth 6 (4 children per survivor): 126 extra is over the limit; depth 5
    # (5 children): 100 extra (107 - 7) is the limit
    assert rule(n, flat, {5: 7}, {9: 501, 6: 126, 5: 107}) == [1, 3, 5, 8]
    assert rule(n, flat, {5: 7}, {9: 501, 6: 126, 5: 108}) == [2, 4, 8]
    # a depth below one that takes the one-machine bound keeps the pair bound
    assert rule(n, flat, {}, {9: 501, 6: 125}) == [2, 4, 6, 8]
    # depths without nodes keep the pair bound (and free the one above)
    assert rule(n, {3: 10, 4: 10}, {}, {}) == [4]
    assert rule(n, {}, {}, {}) == []
    # elim1 above elim2 (not expected) counts as no extra elimination
    assert rule(4, {1: 10, 2: 10, 3: 10}, {3: 9}, {3: 2}) == [1, 3]
    mask = np.zeros(8, np.uint32)
    z = np.zeros(256, np.uint32).ctypes.data_as(ctypes.c_void_p)
    assert L.fsp_bound_choice_rule(0, z, z, z, mask.ctypes.data_as(ctypes.c_void_p)) == -1
    assert L.fsp_bound_choice_rule(10, None, z, z, mask.ctypes.data_as(ctypes.c_void_p)) == -1


def test_model_trained_jobs_rejects_a_null_model(L):
    # argument checks come before any device work
    L.fsp_model_set_trained_jobs.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.fsp_model_set_trained_jobs.restype = ctypes.c_int
    assert L.fsp_model_set_trained_jobs(None, 50) == -1
