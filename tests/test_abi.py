"""CPU-side checks of the C ABI: the library loads without a GPU, exports every
function that include/eecmg.h declares, and the binding's structures have the
C layout."""
import ctypes
import os
import re
import subprocess

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "eecmg.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(eecmg_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    fns = _declared_functions()
    for name in ["eecmg_restore", "eecmg_restore_dev", "eecmg_restore_batch_dev", "eecmg_create", "eecmg_submit",
                 "eecmg_poll", "eecmg_cancel", "eecmg_destroy", "eecmg_last_error", "eecmg_params_default"]:
        assert name in fns


def test_library_exports_every_declared_symbol():
    from paper_2311_03010_amd import eecmg

    lib = ctypes.CDLL(eecmg.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_c(tmp_path):
    from paper_2311_03010_amd import eecmg

    prog = tmp_path / "sz.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "eecmg.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(eecmg_params), sizeof(eecmg_stats),'
                    ' sizeof(eecmg_ctx_config), offsetof(eecmg_params, stats), offsetof(eecmg_stats, final_rms));'
                    'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = [ctypes.sizeof(eecmg.Params), ctypes.sizeof(eecmg.Stats), ctypes.sizeof(eecmg.CtxConfig),
           eecmg.Params.stats.offset, eecmg.Stats.final_rms.offset]
    assert [int(v) for v in out] == got


def test_host_only_entry_points_without_gpu():
    # coarse PSF and parameter defaults never touch the device
    import numpy as np

    import oracle
    from paper_2311_03010_amd import eecmg, synth

    p = eecmg.make_params()
    assert p.precision == 1 and p.stop_rule == 1 and abs(p.c - 1.1) < 1e-15 and p.pm_steps == 1
    for psf in (synth.disk_psf(6), synth.gaussian_psf(3.0, 7)):
        for mode in (0, 1, 2):
            np.testing.assert_allclose(eecmg.coarse_psf(psf, mode), oracle.coarse_psf(psf, mode), rtol=1e-15)
    with pytest.raises(eecmg.EecmgError):
        eecmg.coarse_psf(synth.disk_psf(6), 7)
    # the profiler's pixel filter rejects a negative or NaN bound and accepts 0
    assert eecmg.lib().eecmg_profile_min_pixels(-1.0) == eecmg.EINVAL
    assert eecmg.lib().eecmg_profile_min_pixels(float("nan")) == eecmg.EINVAL
    assert eecmg.lib().eecmg_profile_min_pixels(0.0) == eecmg.OK


def test_fp16_coarse_precision_is_refused_before_any_device_work():
    # the parameters are validated before the device is touched (see
    # test_fp16_coarse_error.py for why the mode is not provided)
    import numpy as np

    from paper_2311_03010_amd import eecmg, synth

    g = np.zeros((64, 64), np.float32)
    with pytest.raises(eecmg.EecmgError) as e:
        eecmg.restore(g, synth.disk_psf(2), 3, precision="f32_f16coarse")
    assert e.value.status == eecmg.EINVAL
    assert "FP16" in str(e.value)
