"""The C ABI on the host: the library loads, exports every declared symbol,
the ctypes structs match the header's layout, and argument validation
returns the documented status codes without touching a GPU."""
import ctypes as C
import os
import re
import subprocess
import sys
import tempfile

import pytest

from paper_1911_10630_amd import exx as X
from paper_1911_10630_amd import synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exx.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(exx_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = X.load()
    names = _declared()
    assert set(names) == set(X.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", X.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, flags=re.M), n


def _c_layout():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "exx.h"
#define O(T, f) printf("%s %zu\n", #f, offsetof(T, f));
#define OS(f) printf("s_%s %zu\n", #f, offsetof(exx_stats_t, f));
int main(void) {
  printf("params %zu\n", sizeof(exx_params));
  O(exx_params, n_grid) O(exx_params, cell) O(exx_params, r_pair) O(exx_params, r_pe) O(exx_params, r_me)
  O(exx_params, fd_half_width) O(exx_params, l_max) O(exx_params, cg_rtol) O(exx_params, cg_max_iter)
  O(exx_params, precision) O(exx_params, orbital_dtype) O(exx_params, guess) O(exx_params, inner_rtol)
  O(exx_params, block_threads) O(exx_params, cg_cols) O(exx_params, wave_pairs) O(exx_params, keep_intermediates)
  O(exx_params, autotune) O(exx_params, graph) O(exx_params, box_dims) O(exx_params, precond)
  O(exx_params, n_classes) O(exx_params, class_r_pe) O(exx_params, class_r_me) O(exx_params, omega_scale)
  printf("stats %zu\n", sizeof(exx_stats_t));
  OS(relres_max) OS(cg_ms) OS(n_pe) OS(n_me) OS(cg_bytes) OS(n_waves) OS(cg_bands) OS(outer_total)
  OS(guess_pairs) OS(guess_ms) OS(tuned) OS(tune_ms) OS(graph_builds) OS(graph_launches) OS(wave_n)
  OS(n_classes) OS(class_n_pe) OS(class_pairs) OS(class_capped)
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "l")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe], text=True)
    return {k: int(v) for k, v in (ln.split() for ln in out.strip().splitlines())}


def test_struct_layout_matches_header():
    lay = _c_layout()
    assert lay["params"] == C.sizeof(X.ExxParams)
    assert lay["stats"] == C.sizeof(X.ExxStats)
    for f in ["n_grid", "cell", "r_pair", "r_pe", "r_me", "fd_half_width", "l_max", "cg_rtol", "cg_max_iter",
              "precision", "orbital_dtype", "guess", "inner_rtol", "block_threads", "cg_cols", "wave_pairs",
              "keep_intermediates", "autotune", "graph", "box_dims", "precond", "n_classes", "class_r_pe",
              "class_r_me", "omega_scale"]:
        assert lay[f] == getattr(X.ExxParams, f).offset, f
    for f in ["relres_max", "cg_ms", "n_pe", "n_me", "cg_bytes", "n_waves", "cg_bands", "outer_total",
              "guess_pairs", "guess_ms", "tuned", "tune_ms", "graph_builds", "graph_launches", "wave_n",
              "n_classes", "class_n_pe", "class_pairs", "class_capped"]:
        assert lay["s_" + f] == getattr(X.ExxStats, f).offset, f


def test_default_params():
    p = X.ExxParams()
    X.load().exx_default_params(C.byref(p))
    assert p.fd_half_width == 3 and p.l_max == 6 and p.cg_rtol == 1e-10 and p.precision == 0
    assert p.autotune == 1


def _setup_status(**over):
    L = X.load()
    p = X.ExxParams()
    L.exx_default_params(C.byref(p))
    wl = S.c1_small()
    for a in range(3):
        p.n_grid[a] = wl.n_grid[a]
        p.cell[a] = wl.cell[a]
    p.r_pair = wl.r_pair
    p.r_pe[0] = p.r_pe[1] = wl.r_pe[0]
    p.r_me[0] = p.r_me[1] = wl.r_me[0]
    for k, v in over.items():
        if isinstance(v, tuple):
            arr = getattr(p, k)
            for i, vv in enumerate(v):
                arr[i] = vv
        else:
            setattr(p, k, v)
    h = C.c_void_p()
    st = L.exx_setup(C.byref(p), 0, C.byref(h))
    msg = L.exx_last_error(None).decode()
    if st == 0:
        L.exx_destroy(h)
    return st, msg


@pytest.mark.parametrize("over,needle", [
    (dict(r_me=(4.0 * S.ANG + 0.5, 4.0 * S.ANG + 0.5)), "n max(h)"),   # shell thinner than the stencil
    (dict(r_pe=(0.0, 1.0)), "r_pe[0]"),
    (dict(fd_half_width=2), "fd_half_width"),
    (dict(l_max=4), "l_max"),
    (dict(precision=7), "precision"),
    (dict(orbital_dtype=3), "orbital_dtype"),
    (dict(cg_rtol=0.0), "cg_rtol"),
    (dict(n_grid=(4, 48, 48)), "n_grid"),
    (dict(box_dims=(49, 0, 0)), "box_dims"),
    (dict(precond=2), "precond"),
    (dict(n_classes=1), "n_classes"),
    (dict(n_classes=5), "n_classes"),
    (dict(n_classes=2, class_r_pe=(3.0, 2.0, 0, 0), class_r_me=(5.0, 4.0, 0, 0), omega_scale=3.0), "ascending"),
    (dict(n_classes=2, class_r_pe=(2.0, 3.0, 0, 0), class_r_me=(2.5, 5.0, 0, 0), omega_scale=3.0), "class_r_me[0]"),
    (dict(n_classes=2, class_r_pe=(2.0, 3.0, 0, 0), class_r_me=(4.0, 5.0, 0, 0), omega_scale=0.0), "omega_scale"),
])
def test_setup_rejects_bad_parameters(over, needle):
    st, msg = _setup_status(**over)
    assert st == X.EXX_EINVAL and needle in msg


def test_setup_null_pointers():
    L = X.load()
    assert L.exx_setup(None, 0, None) == X.EXX_EINVAL
    h = C.c_void_p()
    assert L.exx_setup(None, 0, C.byref(h)) == X.EXX_EINVAL
    assert "NULL" in L.exx_last_error(None).decode()


def test_calls_on_null_context():
    L = X.load()
    assert L.exx_pairs(None, 1, None, None) == X.EXX_EINVAL
    assert L.exx_solve(None, None, None) == X.EXX_EINVAL
    e = C.c_double()
    assert L.exx_energy_potential(None, C.byref(e), None, None) == X.EXX_EINVAL
    assert L.exx_model_init(None, 2, 0) == X.EXX_EINVAL
    assert L.exx_model_train(None, 1, 1, 1e-3, 0, C.byref(e), None) == X.EXX_EINVAL
    n = C.c_size_t()
    assert L.exx_model_save(None, None, C.byref(n)) == X.EXX_EINVAL
    assert L.exx_load_model(None, None, 0) == X.EXX_EINVAL
    assert L.exx_model_conv(None, 0, 0, None, None, 1, 1, None) == X.EXX_EINVAL
    assert L.exx_model_wgrad(None, 0, None, None, None, 1, 1, None) == X.EXX_EINVAL
    assert L.exx_model_edge(None) == 0
    L.exx_destroy(None)


def test_learned_guess_is_a_valid_mode():
    """guess = EXX_GUESS_LEARNED passes validation (and fails only for the
    missing device here); one past it is rejected."""
    st, msg = _setup_status(guess=4)
    assert st == X.EXX_EINVAL and "guess" in msg
    st, msg = _setup_status(guess=3)
    assert st != X.EXX_EINVAL


def test_setup_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, msg = _setup_status()
    assert st == X.EXX_EDEVICE and "device" in msg


def test_host_allocation_failure_is_a_status():
    """A host allocation that fails inside the library comes back through the
    C ABI as EXX_ENOMEM with a message, never as a C++ exception (which would
    terminate the caller): exx_setup under an address-space limit, asked for
    a PE sphere of about 8e7 points whose tables cannot fit.  The tables are
    built before any device call, so this runs without a GPU."""
    import subprocess
    code = r"""
import ctypes as C, resource, sys
sys.path.insert(0, %r)
from paper_1911_10630_amd import exx as X
L = X.load()
p = X.ExxParams()
L.exx_default_params(C.byref(p))
for a in range(3):
    p.n_grid[a] = 600
    p.cell[a] = 600.0
p.r_pair = 1.0
p.r_pe[0] = p.r_pe[1] = 270.0
p.r_me[0] = p.r_me[1] = 274.0
vm = [int(l.split()[1]) for l in open('/proc/self/status') if l.startswith('VmSize')][0] * 1024
resource.setrlimit(resource.RLIMIT_AS, (vm + (256 << 20), resource.RLIM_INFINITY))
h = C.c_void_p()
st = L.exx_setup(C.byref(p), 0, C.byref(h))
resource.setrlimit(resource.RLIMIT_AS, (resource.RLIM_INFINITY, resource.RLIM_INFINITY))
print(st)
print(L.exx_last_error(None).decode())
""" % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    st, msg = out.stdout.strip().splitlines()[-2:]
    assert int(st) == X.EXX_ENOMEM and "exx_setup: host allocation failed" in msg, (st, msg)
