"""The C-ABI library loads and exports every entry point include/tk.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_11404_amd", "libtk.so")


def declared():
    text = open(os.path.join(ROOT, "include", "tk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tk_[a-z0-9_]+)\s*\(", text)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtk.so not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (binds torch's HIP runtime first, as the binding does)
    L = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 16
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtk.so not built")
def test_host_only_entry_points():
    from paper_2603_11404_amd import tk
    L = tk.lib()
    assert L.tk_version() == 100
    assert L.tk_status_string(1) == b"TK_ERR_INVALID_ARGUMENT"
    assert tk.cmaes_state_bytes(9, 16) > 0 and tk.cmaes_state_bytes(9, 16) % 256 == 0
    assert tk.cmaes_state_bytes(0, 16) == 0 and tk.cmaes_state_bytes(19, 16) == 0
    assert tk.cmaes_state_bytes(9, 1025) == 0
    lay = tk.cmaes_layout(18, 1024)
    assert lay["order"] + 4 * 1024 <= lay["total_bytes"]
    with pytest.raises(tk.TkError) as e:
        tk.cmaes_layout(0, 16)
    assert e.value.status == 1


def test_binding_exports_match_header():
    from paper_2603_11404_amd import tk
    assert sorted(tk.EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtk.so not built")
def test_filter_argument_errors_launch_nothing():
    """tk_kf_init rejects bad parameters on the host before any launch."""
    import numpy as np
    from paper_2603_11404_amd import tk
    assert tk.lib().tk_kf_state_bytes(9) >= 9 * 11 * 8 and tk.lib().tk_kf_state_bytes(19) == 0
    assert tk.lib().tk_kf_state_bytes(0) == 0
    good = dict(n=3, dt=1.0, p0_pos=1.0, p0_vel=1.0, q_pos=1e-4, q_vel=1e-4, r=1e-2)
    fake = ctypes.c_void_p(256)           # never dereferenced: every case below fails validation
    for bad in (dict(dt=0.0), dict(r=0.0), dict(q_pos=-1.0), dict(q_cross=1.0), dict(p0_vel=np.nan),
                dict(lo=1.0, hi=0.0)):
        p = tk.kf_params(**{**good, **bad})
        st = tk.lib().tk_kf_init(fake, 3, np.zeros(3).ctypes.data_as(ctypes.c_void_p), ctypes.byref(p), None)
        assert st == 1, bad
    p = tk.kf_params(**good, lo=0.5, hi=1.0)          # x0 = 0 outside the clamp limits
    assert tk.lib().tk_kf_init(fake, 3, np.zeros(3).ctypes.data_as(ctypes.c_void_p), ctypes.byref(p), None) == 1
    assert tk.lib().tk_kf_step(fake, 0, fake, None, None, None) == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtk.so not built")
def test_soft_and_adam_argument_errors_launch_nothing():
    """Sizes and argument checks of the differentiable form run on the host
    before any launch (fake device addresses are never dereferenced)."""
    import numpy as np
    import scenes
    from paper_2603_11404_amd import tk
    L = tk.lib()
    wl = scenes.workload("soft640")
    m = wl["mesh"]
    fake = 1 << 20
    meshes = (tk.Mesh * 1)(tk.Mesh(m.n_vertices, m.n_triangles, fake, fake, fake))
    cam = tk.camera(wl["cam"])
    nb = L.tk_soft_workspace_bytes(256, meshes, 1, ctypes.byref(cam))
    # corners, face records, tile lists (32 per face), big list, G, partials
    assert nb >= 256 * (m.n_vertices * 16 + m.n_triangles * (48 + 32 * 4 + 4) + 640 * 480 * 4)
    assert L.tk_soft_workspace_bytes(512, meshes, 1, ctypes.byref(cam)) > nb
    big = tk.camera(scenes.camera(2048, 2048))
    assert L.tk_soft_workspace_bytes(1, meshes, 1, ctypes.byref(big)) == 0       # over 16384 tiles
    assert L.tk_soft_workspace_bytes(1, meshes, 3, ctypes.byref(cam)) == 0       # three arms
    p = ctypes.c_void_p(fake)
    assert L.tk_soft_forward(p, 1, meshes, 1, ctypes.byref(cam), ctypes.c_float(0.0), p, None, p, p,
                             ctypes.c_size_t(nb), None) == tk.TK_ERR_INVALID_ARGUMENT
    assert L.tk_soft_forward(p, 1, meshes, 1, ctypes.byref(big), ctypes.c_float(1.0), p, None, p, p,
                             ctypes.c_size_t(nb), None) == tk.TK_ERR_UNSUPPORTED
    assert L.tk_soft_forward(p, 256, meshes, 1, ctypes.byref(cam), ctypes.c_float(1.0), p, None, p, p,
                             ctypes.c_size_t(nb - 1), None) == tk.TK_ERR_WORKSPACE_TOO_SMALL
    assert L.tk_soft_forward(p, 256, meshes, 1, ctypes.byref(cam), ctypes.c_float(1.0), p, None, p,
                             ctypes.c_void_p(fake + 8), ctypes.c_size_t(nb + 64), None) == tk.TK_ERR_INVALID_ARGUMENT
    assert L.tk_adam_reset(p, 0, None) == tk.TK_ERR_INVALID_ARGUMENT
    for lr, b1, b2, eps in [(0.0, 0.9, 0.999, 1e-8), (0.1, 1.0, 0.999, 1e-8), (0.1, 0.9, 0.999, 0.0)]:
        assert L.tk_cmaes_adam(p, 9, 16, p, p, lr, b1, b2, eps, None) == tk.TK_ERR_INVALID_ARGUMENT


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtk.so not built")
def test_init_at_argument_errors_launch_nothing():
    """tk_cmaes_init_at checks sizes, pointers, readings and joint limits on
    the host before any launch (fake device addresses are never dereferenced)."""
    import numpy as np
    import scenes
    from paper_2603_11404_amd import tk
    L = tk.lib()
    p = ctypes.c_void_p(1 << 20)
    good = tk.chain(scenes.chain())
    ch = (tk.Chain * 2)(good, good)
    sc = np.ones(18)
    par = tk.CmaesParams(1.0, 1.0, 1.0, 1)

    def call(n=18, est=p, chains=ch, n_arms=2, readings=None, sigma0=1.0):
        r = None if readings is None else np.ascontiguousarray(readings, np.float64).ctypes.data_as(ctypes.c_void_p)
        return L.tk_cmaes_init_at(p, n, 16, est, chains, n_arms, r, sigma0, sc.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(par), 1, None)
    bad = tk.chain(scenes.chain())
    bad.q_lb[1], bad.q_ub[1] = 0.5, 0.5
    assert call(n=9) == tk.TK_ERR_INVALID_ARGUMENT                      # n != 9 x n_arms
    assert call(est=None) == tk.TK_ERR_INVALID_ARGUMENT
    assert call(readings=[0, 0, np.nan, 0, 0, 0]) == tk.TK_ERR_INVALID_ARGUMENT
    assert call(chains=(tk.Chain * 2)(good, bad)) == tk.TK_ERR_INVALID_ARGUMENT
    assert call(sigma0=0.0) == tk.TK_ERR_INVALID_ARGUMENT
    assert call(n_arms=3, n=27) == tk.TK_ERR_INVALID_ARGUMENT           # more arms than supported
