"""Host-side check of the pass launches' arguments (no GPU): every launch of
a solve's Newton loop and every autotuner trial launch carries the operands
its mode reads, for the workloads' shapes; an omission planted in one of the
tuner's launches (the kind of dropped argument line that once sent null
pointers to a CG-update launch) is caught and named.  The same checks run
under AddressSanitizer and UndefinedBehaviorSanitizer on a host-sanitised
build of the library when that build is present (python -m
paper_1301_1215_amd.build --sanitize)."""
import os
import subprocess
import sys

import pytest

from paper_1301_1215_amd import _native as N

SHAPES = [(64, 64, 8, 1), (384, 192, 12, 4), (512, 256, 32, 1), (96, 40, 4, 2), (12, 12, 2, 1), (192, 96, 6, 3)]
COL_MODES = {0: "col_winv_ifft", 7: "col_pupd_winv_ifft", 1: "col_p_ifft", 2: "col_fft_p", 3: "col_resid_p_ifft",
             4: "col_psf", 5: "col_fft_winv_add", 8: "col_fft_winv_cg_update"}


def _coil_maps_go_on_into_the_forward(n, m):
    """Omega the centred half on compile-time slots of the line split: the
    coil-map row pass also does the forward model's row pass."""
    n1 = max(d for d in range(1, n + 1) if d * d <= n and n % d == 0 and d <= 32 and n // d <= 32)
    n2 = n // n1
    return 2 * m == n and n1 % 2 == 0 and n2 % 4 == 0 and (n // 4) % n1 == 0


@pytest.mark.parametrize("n,m,J,F", SHAPES)
def test_every_launch_carries_its_operands(n, m, J, F):
    st, cnt, bad = N.nlinv_check_launch_args(n, m, J, F, newton=3, cg=4)
    assert st == N.NLINV_OK and bad == -1
    # per Newton step: coil maps (2), residual (2; 1 where the coil-map row
    # pass goes on into the forward model's), right-hand side (3), 5 per CG
    # iteration; the final coil maps (2); the tuner's 8 column and 4 row
    # launches, and on grids up to 64 its whole-plane normal operator with its
    # coil sum (2) and a whole-plane CG iteration (2)
    resid = 1 if _coil_maps_go_on_into_the_forward(n, m) else 2
    assert cnt == 3 * (2 + resid + 3 + 5 * 4) + 2 + 8 + 4 + (4 if n <= 64 else 0)


@pytest.mark.parametrize("mode", sorted(COL_MODES))
def test_a_dropped_argument_is_caught(mode):
    st, cnt, bad = N.nlinv_check_launch_args(384, 192, 12, 2, drop_mode=mode)
    assert st == N.NLINV_EINVAL
    assert N.nlinv_kernel_class_names()[bad] == COL_MODES[mode]


def test_under_address_and_undefined_behaviour_sanitizers():
    lib = os.path.join(os.path.dirname(N.LIB_PATH), "libnlinv_san.so")
    if not os.path.exists(lib):
        pytest.skip("host-sanitised build absent (python -m paper_1301_1215_amd.build --sanitize)")
    from paper_1301_1215_amd.build import asan_runtime
    code = ("import ctypes, sys; sys.path.insert(0, %r); from paper_1301_1215_amd import _native as N; "
            "lib = N.load(%r); "
            "r = [N.nlinv_check_launch_args(n, m, J, F, 2, 3, -1, lib) for n, m, J, F in %r]; "
            "assert all(x[0] == 0 and x[2] == -1 for x in r), r; "
            "assert N.nlinv_check_launch_args(384, 192, 12, 1, 1, 1, 8, lib)[0] == -1; print('sanitized ok')"
            % (os.path.dirname(os.path.dirname(N.LIB_PATH)), lib, SHAPES))
    env = dict(os.environ, LD_PRELOAD=asan_runtime(), ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "sanitized ok" in r.stdout, r.stdout + r.stderr
