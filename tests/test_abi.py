"""Host-side checks of the C ABI: the library loads, exports every function
include/helios.h declares, its structs have the layout the C compiler gives
them, and argument validation rejects bad calls before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "helios.h")


@pytest.fixture(scope="module")
def H():
    from paper_1606_05474_amd import helios

    if not os.path.exists(helios.LIB_PATH):
        from paper_1606_05474_amd import build

        build.build()
    helios.lib()
    return helios


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(helios_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_function_is_exported(H):
    names = declared_functions()
    assert {"helios_mix_opacity", "helios_flux", "helios_radeq", "helios_grid", "helios_profile",
            "helios_transmission", "helios_workspace_bytes", "helios_last_error", "helios_version"} <= set(names)
    lib = H.lib()
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", H.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n


def test_struct_layouts_match_the_c_compiler(tmp_path, H):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "helios.h"
#define P(T, f) printf(#T "." #f " %zu\\n", offsetof(T, f));
int main(void) {
  printf("helios_atm %zu\\n", sizeof(helios_atm));
  printf("helios_ktab %zu\\n", sizeof(helios_ktab));
  printf("helios_re_opts %zu\\n", sizeof(helios_re_opts));
  printf("helios_re_state %zu\\n", sizeof(helios_re_state));
  printf("helios_mlp %zu\\n", sizeof(helios_mlp));
  P(helios_mlp, params) P(helios_mlp, out_scale)
  P(helios_atm, T_int) P(helios_atm, status) P(helios_atm, P_pt) P(helios_ktab, k) P(helios_ktab, mmw) P(helios_ktab, species_mass)
  P(helios_re_opts, T_floor) P(helios_re_opts, fpre_p) P(helios_re_state, iter)
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)], text=True).splitlines())
    assert int(got["helios_atm"]) == ctypes.sizeof(H.HeliosAtm)
    assert int(got["helios_ktab"]) == ctypes.sizeof(H.HeliosKtab)
    assert int(got["helios_re_opts"]) == ctypes.sizeof(H.HeliosReOpts)
    assert int(got["helios_re_state"]) == ctypes.sizeof(H.HeliosReState)
    assert int(got["helios_mlp"]) == ctypes.sizeof(H.HeliosMlp)
    assert int(got["helios_mlp.params"]) == H.HeliosMlp.params.offset
    assert int(got["helios_mlp.out_scale"]) == H.HeliosMlp.out_scale.offset
    assert int(got["helios_atm.T_int"]) == H.HeliosAtm.T_int.offset
    assert int(got["helios_atm.status"]) == H.HeliosAtm.status.offset
    assert int(got["helios_atm.P_pt"]) == H.HeliosAtm.P_pt.offset
    assert int(got["helios_ktab.k"]) == H.HeliosKtab.k.offset
    assert int(got["helios_ktab.mmw"]) == H.HeliosKtab.mmw.offset
    assert int(got["helios_ktab.species_mass"]) == H.HeliosKtab.species_mass.offset
    assert int(got["helios_re_opts.T_floor"]) == H.HeliosReOpts.T_floor.offset
    assert int(got["helios_re_opts.fpre_p"]) == H.HeliosReOpts.fpre_p.offset
    assert int(got["helios_re_state.iter"]) == H.HeliosReState.iter.offset


def test_validation_rejects_bad_descriptors_without_a_device(H):
    import numpy as np

    lib = H.lib()
    assert lib.helios_grid(None, None) == -1
    assert b"NULL" in lib.helios_last_error()
    n_layer = np.array([1], np.int32)   # fewer than 2 layers
    n_bin = np.array([3], np.int32)
    fake = ctypes.c_void_p(16)           # never dereferenced: validation fails first
    d = H.HeliosAtm(1, 20, n_layer.ctypes.data, n_bin.ctypes.data, *([fake] * 17))
    assert lib.helios_grid(ctypes.byref(d), None) == -2
    assert b"n_layer" in lib.helios_last_error()
    d.n_g = 0
    assert lib.helios_grid(ctypes.byref(d), None) == -1
    d.n_g = 20
    n_layer[0] = 50
    n_bin[0] = 0
    assert lib.helios_profile(ctypes.byref(d), fake, fake, None) == -2
    n_bin[0] = 3
    assert lib.helios_workspace_bytes(ctypes.byref(d), 0) > 0
    assert lib.helios_workspace_bytes(ctypes.byref(d), 1) <= lib.helios_workspace_bytes(ctypes.byref(d), 0)
    kt = H.HeliosKtab()
    kt.mode = 7
    assert lib.helios_mix_opacity(ctypes.byref(d), ctypes.byref(kt), fake, fake, fake, 0, None) == -1
    kt.mode = 0
    kt.n_species = 1
    kt.n_g = 19
    assert lib.helios_mix_opacity(ctypes.byref(d), ctypes.byref(kt), fake, fake, fake, 0, None) == -2
    assert lib.helios_mix_opacity(ctypes.byref(d), ctypes.byref(kt), fake, fake, fake, 5, None) == -1
    opts = H.REOptions(window=1).c()
    st = H.HeliosReState(fake, fake, None)
    assert lib.helios_radeq(ctypes.byref(d), fake, fake, fake, ctypes.byref(st), ctypes.byref(opts), fake,
                            None, None) == -1
    assert lib.helios_version() >= 1


def test_mode_entry_points_validate_before_any_device_work(H):
    """helios_flux_iso and helios_flux_rayleigh reject bad arguments on the
    host (nothing is enqueued); the layer limit is the long-column shape's."""
    import numpy as np

    lib = H.lib()
    n_layer = np.array([50], np.int32)
    n_bin = np.array([3], np.int32)
    fake = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    d = H.HeliosAtm(1, 20, n_layer.ctypes.data, n_bin.ctypes.data, *([fake] * 17))
    args = (fake, fake, fake, fake, 4, 2.0, fake, None, None, None, fake, fake, 1 << 30, 0, None)
    assert lib.helios_flux_iso(ctypes.byref(d), None, *args[1:]) == -1  # NULL opacities
    assert lib.helios_flux_iso(ctypes.byref(d), fake, fake, fake, fake, 4, 2.0, fake, None, None, None, None,
                               fake, 1 << 30, 0, None) == -1  # NULL F_bol
    assert lib.helios_flux_rayleigh(ctypes.byref(d), fake, fake, 0.0, 4, 2.0, fake, None, None, None, fake, fake,
                                    1 << 30, 0, None) == -1
    assert b"mbar" in lib.helios_last_error()
    assert lib.helios_flux_rayleigh(ctypes.byref(d), None, fake, 4e-24, 4, 2.0, fake, None, None, None, fake,
                                    fake, 1 << 30, 0, None) == -1
    assert lib.helios_flux_rayleigh(ctypes.byref(d), fake, fake, 4e-24, -1, 2.0, fake, None, None, None, fake,
                                    fake, 1 << 30, 0, None) == -1  # negative scattering-pass count
    n_layer[0] = 833
    assert lib.helios_grid(ctypes.byref(d), None) == -2
    assert b"2..832" in lib.helios_last_error()
    n_layer[0] = 832
    assert lib.helios_workspace_bytes(ctypes.byref(d), 0) > 0


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with status 2 and
    says why, before touching a device."""
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
