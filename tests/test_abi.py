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
  P(helios_atm, T_int) P(helios_atm, status) P(helios_atm, P_pt) P(helios_atm, bin_index_h) P(helios_ktab, k) P(helios_ktab, mmw) P(helios_ktab, species_mass)
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
    assert int(got["helios_atm.bin_index_h"]) == H.HeliosAtm.bin_index_h.offset
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
    d = H.HeliosAtm(1, 20, n_layer.ctypes.data, n_bin.ctypes.data, *([fake] * 18))
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
    d = H.HeliosAtm(1, 20, n_layer.ctypes.data, n_bin.ctypes.data, *([fake] * 18))
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
    n_layer[0] = 1025
    assert lib.helios_grid(ctypes.byref(d), None) == -2
    assert b"2..1024" in lib.helios_last_error()
    n_layer[0] = 1024
    assert lib.helios_workspace_bytes(ctypes.byref(d), 0) > 0


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with status 2 and
    says why, before touching a device."""
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _desc(H, n=50, nb=3, bin_index=None):
    """A descriptor whose device pointers are never dereferenced (validation
    fails first) and whose host mirrors are real arrays."""
    import numpy as np

    fake = ctypes.c_void_p(16)
    keep = {"n_layer": np.array([n], np.int32), "n_bin": np.array([nb], np.int32),
            "bin_index": np.ascontiguousarray(np.arange(nb) if bin_index is None else bin_index, np.int32)}
    d = H.HeliosAtm(1, 20, keep["n_layer"].ctypes.data, keep["n_bin"].ctypes.data, *([fake] * 18))
    d.bin_index_h = keep["bin_index"].ctypes.data
    return d, keep, fake


def test_mix_opacity_rejects_a_bin_outside_the_table(H):
    """A model bin whose table index lies outside the table (Sec. 2.3 looks
    up the k-distribution of the bin) is -2 with nothing enqueued, checked on
    the host mirror of bin_index."""
    import numpy as np

    lib = H.lib()
    mass = np.array([18.0], np.float64)
    kt = H.HeliosKtab(H.KTAB_TABLE, 1, 2, 2, 3, 20, 100.0, 100.0, 0.0, 1.0, ctypes.c_void_p(16), None, 0.0, 0.0,
                      1.0, 1.0, mass.ctypes.data, 2.4)
    for bad in ([0, 1, 3], [0, -1, 2]):
        d, keep, fake = _desc(H, bin_index=bad)
        assert lib.helios_mix_opacity(ctypes.byref(d), ctypes.byref(kt), fake, fake, fake, 0, None) == -2
        assert b"bin_index" in lib.helios_last_error()
    d, keep, fake = _desc(H, bin_index=[0, 1, 2])
    kt.mmw = 0.0  # the bins are fine now: the next check (masses) fails instead
    assert lib.helios_mix_opacity(ctypes.byref(d), ctypes.byref(kt), fake, fake, fake, 0, None) == -1
    d.bin_index_h = None
    assert lib.helios_mix_opacity(ctypes.byref(d), ctypes.byref(kt), fake, fake, fake, 0, None) == -1


def test_state_flags_and_conversion_validate_on_the_host(H):
    """The per-g convention flag is accepted in a flux call's prec argument
    and nowhere else; unknown flags, modes and layers are -1 before any
    device work."""
    lib = H.lib()
    d, keep, fake = _desc(H)
    big = 1 << 40
    args = lambda prec: (ctypes.byref(d), fake, fake, fake, fake, 4, 2.0, fake, None, None, None, fake, fake,  # noqa
                         big, prec, None)
    assert lib.helios_flux(*args(0x200)) == -1 and b"flags" in lib.helios_last_error()
    assert lib.helios_flux(*args(H.FP64 | H.STATE_FLUX | 0x400)) == -1
    assert lib.helios_workspace_bytes(ctypes.byref(d), H.MIXED | H.STATE_FLUX) == \
        lib.helios_workspace_bytes(ctypes.byref(d), H.MIXED)
    assert lib.helios_state_convert(ctypes.byref(d), fake, 2.0, fake, 3, 0, 0, None) == -1
    assert lib.helios_state_convert(ctypes.byref(d), fake, 2.0, fake, 0, 2, 0, None) == -1
    assert lib.helios_state_convert(ctypes.byref(d), fake, 0.0, fake, 0, 0, 0, None) == -1
    assert lib.helios_state_convert(ctypes.byref(d), None, 2.0, fake, 0, 0, 0, None) == -1
    assert lib.helios_state_convert(ctypes.byref(d), fake, 2.0, fake, 0, 0, H.FP64 | H.STATE_FLUX, None) == -1
    assert lib.helios_flux_exact(ctypes.byref(d), fake, fake, fake, fake, None, None, fake, fake, big, 0x300,
                                 None) == -1
    out = (ctypes.c_int32 * 18)()
    assert lib.helios_sweep_shapes(ctypes.byref(d), 0, out, 5) == -1  # six classes need room for six
    assert lib.helios_sweep_shapes(ctypes.byref(d), H.MIXED | H.STATE_FLUX, out, 6) == 6


def test_autotune_reset_returns_to_the_default_shapes(H):
    """helios_autotune_reset is host-only and always succeeds; afterwards
    helios_sweep_shapes reports the default shapes."""
    lib = H.lib()
    d, keep, fake = _desc(H, n=100)
    out = (ctypes.c_int32 * 18)()
    assert lib.helios_autotune_reset() == 0
    assert lib.helios_sweep_shapes(ctypes.byref(d), 0, out, 6) == 6
    # 100 layers (200 sublayers): class n <= 112, fewest sublayers per lane that hold them
    assert (out[3 * 2], out[3 * 2 + 1], out[3 * 2 + 2]) == (112, 8, 32)
