"""The C ABI: library loads, exports every declared symbol, the ctypes mirror of
the structs matches the C layout, and invalid configurations are rejected on
the host (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ulmproj.h")


def _lib():
    from paper_2511_21647_amd import _lib as L
    return L


def test_library_exports_every_declared_symbol():
    L = _lib()
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:const\s+char\s*\*|int32_t)\s*(\w+)\s*\(", text, re.M))
    assert declared == set(L.EXPORTS)
    raw = ctypes.CDLL(L.LIB_PATH)
    for name in declared:
        assert hasattr(raw, name), name


def test_struct_layout_matches_header(tmp_path):
    L = _lib()
    src = tmp_path / "layout.c"
    fields = [f[0] for f in L.ULMConfig._fields_]
    body = "\n".join(f'printf("%s %zu\\n", "{f}", offsetof(ulm_config_t, {f}));' for f in fields)
    loc_fields = list(L.LOC_DTYPE.names)
    body += "\n" + "\n".join(f'printf("loc.%s %zu\\n", "{f}", offsetof(ulm_loc_t, {f}));'
                             for f in loc_fields)
    src.write_text(f"""#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
{body}
printf("sizeof_config %zu\\n", sizeof(ulm_config_t));
printf("sizeof_loc %zu\\n", sizeof(ulm_loc_t));
printf("sizeof_timing %zu\\n", sizeof(ulm_timing_t));
return 0; }}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for f in fields:
        assert int(out[f]) == getattr(L.ULMConfig, f).offset, f
    for f in loc_fields:
        assert int(out["loc." + f]) == L.LOC_DTYPE.fields[f][1], f
    assert int(out["sizeof_config"]) == ctypes.sizeof(L.ULMConfig)
    assert int(out["sizeof_loc"]) == L.LOC_DTYPE.itemsize
    assert int(out["sizeof_timing"]) == ctypes.sizeof(L.ULMTiming)


def _create(cfg_struct):
    L = _lib()
    h = ctypes.c_void_p()
    rc = L._lib.ulm_create(ctypes.byref(cfg_struct), ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("mutate,msg", [
    (lambda c: setattr(c, "n_angles", 0), "n_angles"),
    (lambda c: setattr(c, "n_angles", 33), "n_angles"),
    (lambda c: setattr(c, "ncc_size", 8), "ncc_size"),
    (lambda c: setattr(c, "ncc_size", 17), "ncc_size"),
    (lambda c: setattr(c, "svd_cutoff", 33), "svd_cutoff"),
    (lambda c: setattr(c, "svd_cutoff", -1), "svd_cutoff"),
    (lambda c: setattr(c, "n_frames", 2000), "n_frames"),
    (lambda c: setattr(c, "pitch", 0.0), "physical"),
    (lambda c: setattr(c, "precision", 7), "precision"),
    (lambda c: setattr(c, "n_blocks", 0), "grid"),
    (lambda c: setattr(c, "nu", 4000), "NCC band"),
    (lambda c: setattr(c, "z0", -1e-3), "z0"),
    (lambda c: setattr(c, "n_samp", 4), "n_samp"),
])
def test_invalid_config_rejected_on_host(mutate, msg):
    from synth import cfg_paper
    L = _lib()
    c = L.make_config(cfg_paper())
    mutate(c)
    rc, h = _create(c)
    assert rc == L.ULM_ERR_INVALID_ARG
    assert msg in L.last_error()
    assert not h.value


def test_delay_span_too_large_rejected():
    """A grid whose tile delay span exceeds the staged sample window is refused."""
    from synth import cfg_paper
    L = _lib()
    c = L.make_config(cfg_paper())
    c.dz = 2e-3                     # 8 rows x 2 mm = a 14 mm tile: far beyond the window
    rc, _ = _create(c)
    assert rc == L.ULM_ERR_INVALID_ARG and "window" in L.last_error()


def test_null_arguments():
    L = _lib()
    assert L._lib.ulm_create(None, None) == L.ULM_ERR_INVALID_ARG
    n = ctypes.c_size_t()
    assert L._lib.ulm_workspace_size(None, ctypes.byref(n)) == L.ULM_ERR_INVALID_ARG
    assert L._lib.rca_beamform_proj(None, None, None, None, 0, None) == L.ULM_ERR_INVALID_ARG
    assert L._lib.svd_clutter_filter(None, None, None, None, 0, None) == L.ULM_ERR_INVALID_ARG
    assert L._lib.ncc_localize(None, None, None, 0, None, None, 0, None) == L.ULM_ERR_INVALID_ARG
    assert L._lib.ulm_destroy(None) == L.ULM_OK


def test_paper_geometry_fits_window():
    """The paper-scale and tiny configurations pass validation up to the first HIP
    call (which fails without a GPU, or succeeds with one)."""
    from synth import cfg_paper, cfg_tiny
    L = _lib()
    for cfg in (cfg_paper(), cfg_tiny()):
        rc, h = _create(L.make_config(cfg))
        assert rc in (L.ULM_OK, L.ULM_ERR_HIP), L.last_error()
        if rc == L.ULM_OK:
            L._lib.ulm_destroy(h)


def test_cnn_arguments_checked_on_host():
    """CNN entry points reject bad sizes, precisions, NULL pointers and short or
    misaligned workspaces before any device work."""
    L = _lib()
    lib, E = L._lib, L.ULM_ERR_INVALID_ARG
    n = ctypes.c_size_t()
    assert lib.ulm_cnn_workspace_size(0, 10, 10, L.ULM_CNN_BF16, 0, ctypes.byref(n)) == E
    assert lib.ulm_cnn_workspace_size(1, 10, 10, 7, 0, ctypes.byref(n)) == E
    assert lib.ulm_cnn_workspace_size(4096, 256, 256, L.ULM_CNN_BF16, 1, ctypes.byref(n)) == E
    assert lib.ulm_cnn_workspace_size(2, 21, 37, L.ULM_CNN_BF16, 1, None) == E
    assert lib.ulm_cnn_workspace_size(2, 21, 37, L.ULM_CNN_BF16, 0, ctypes.byref(n)) == L.ULM_OK
    infer = n.value
    assert lib.ulm_cnn_workspace_size(2, 21, 37, L.ULM_CNN_BF16, 1, ctypes.byref(n)) == L.ULM_OK
    assert n.value > infer
    assert lib.ulm_cnn_workspace_size(2, 21, 37, L.ULM_CNN_FP32, 1, ctypes.byref(n)) == L.ULM_OK
    fake = ctypes.c_void_p(1 << 20)               # never dereferenced: checks fail first
    assert lib.ulm_cnn_forward(None, fake, 2, 21, 37, 0, fake, fake, 1 << 30, None) == E
    assert lib.ulm_cnn_forward(fake, fake, 2, 21, 37, 0, fake, fake, 16, None) == E
    assert "too small" in L.last_error()
    assert lib.ulm_cnn_forward(fake, fake, 2, 21, 37, 0, fake, ctypes.c_void_p((1 << 20) + 8),
                               1 << 30, None) == E
    assert "aligned" in L.last_error()
    assert lib.ulm_cnn_gradients(fake, fake, 2, 21, 37, None, None, 3, 0, fake, fake, fake,
                                 1 << 30, None) == E
    assert lib.ulm_cnn_train_step(fake, fake, fake, 0, ctypes.c_float(1e-3), fake, 2, 21, 37,
                                  None, None, 0, 0, fake, fake, 1 << 30, None) == E
    assert lib.ulm_cnn_localize(None, fake, fake, ctypes.c_float(0.5), 8, 0, fake, 10, fake, fake,
                                1 << 30, fake, 1 << 30, None) == E
    assert lib.ulm_cnn_images(None, fake, fake, fake, 1 << 30, None) == E
    assert lib.ulm_cnn_localize_workspace_size(None, 8, 0, ctypes.byref(n)) == E


def test_cnn_parameter_packing_roundtrip():
    """The flat parameter order is w0, b0, w1, b1, ..., w5, b5, wh, bh."""
    import numpy as np
    L = _lib()
    flat = np.arange(L.ULM_CNN_PARAMS, dtype=np.float32)
    d = L.cnn_unpack(flat)
    assert d["w0"].shape == (32, 1, 3, 3) and d["w0"][1, 0, 2, 1] == 9 + 2 * 3 + 1
    assert d["b0"][0] == 288 and d["w1"][0, 0, 0, 0] == 320
    assert d["bh"][-1] == L.ULM_CNN_PARAMS - 1
    assert np.array_equal(L.cnn_pack(d), flat)
