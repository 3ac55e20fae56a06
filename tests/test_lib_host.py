"""Host-side checks of libboa (no GPU needed): every symbol include/boa.h
declares is exported, and the error paths that need no device behave."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2511_11337_amd", "libboa.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libboa.so not built")


def declared_functions():
    hdr = open(os.path.join(ROOT, "include", "boa.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(boa_[a-z0-9_]+)\s*\(", hdr)))


def test_every_declared_symbol_is_exported():
    from paper_2511_11337_amd import _lib
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    # the ctypes table covers exactly the declared ABI
    assert set(names) == set(_lib.SIGNATURES)


def test_param_count_matches_layout():
    from paper_2511_11337_amd import Config
    from synth import ModelConfig, param_count
    for d, l in [(64, 2), (256, 3), (512, 4), (128, 1)]:
        assert Config(d, l).n_params == param_count(ModelConfig(d, l))
    # unsupported shapes report 0
    assert Config(96, 2).n_params == 0


def test_container_errors_without_device():
    from paper_2511_11337_amd import _lib, container_info, BoaError
    with pytest.raises(BoaError) as e:
        container_info(b"not a container" * 8)
    assert e.value.name == "BOA_E_FORMAT"
    with pytest.raises(BoaError) as e:
        container_info(b"\x00" * 10)
    assert e.value.name == "BOA_E_FORMAT"


def test_numerics_id_encodes_dtype():
    from paper_2511_11337_amd import numerics_id
    assert numerics_id("f32") != numerics_id("bf16")
    assert numerics_id("f32") & 0xFF == 0 and numerics_id("bf16") & 0xFF == 1


def test_model_create_without_gpu_is_an_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2511_11337_amd import Model, Config, BoaError
    from synth import ModelConfig, init_weights
    w = init_weights(ModelConfig(64, 2), 1)
    with pytest.raises(BoaError) as e:
        Model(Config(64, 2), w)
    assert e.value.name in ("BOA_E_UNSUPPORTED", "BOA_E_DEVICE")


def test_bad_config_rejected():
    from paper_2511_11337_amd import _lib
    lib = _lib.load()
    c = _lib.boa_config(64, 2, 8, 4, 2)       # d_state 8 unsupported
    h = C.c_void_p()
    w = np.zeros(10, np.float32)
    rc = lib.boa_model_create(C.byref(c), w.ctypes.data, w.size, 0, C.byref(h))
    assert rc == -1


def _struct_fields(name):
    hdr = open(os.path.join(ROOT, "include", "boa.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + ";", hdr).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, names = decl.split(None, 1)
        fields += [n.strip() for n in names.split(",")]
    return fields


def test_ctypes_structs_match_header():
    """The binding's structs list the header's fields in order (an ABI drift
    would pass garbage options silently)."""
    from paper_2511_11337_amd import _lib
    for cname, ct in [("boa_config", _lib.boa_config), ("boa_run_opts", _lib.boa_run_opts)]:
        assert [f[0] for f in ct._fields_] == _struct_fields(cname), cname
