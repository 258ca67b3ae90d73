"""The C-ABI library loads on a CPU-only host and exports every declared symbol."""
import ctypes
import os
import re

import pytest

from conftest import ROOT


def _declared():
    text = open(os.path.join(ROOT, "include", "bytestore.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bst_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(built_lib):
    names = _declared()
    assert len(names) >= 30
    L = ctypes.CDLL(built_lib)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header(built_lib):
    from paper_2209_00220_amd import _lib

    assert set(_declared()) == set(_lib.exported_names())


def test_library_loads_without_gpu(built_lib):
    from paper_2209_00220_amd import _lib

    assert _lib.bst_version() >= 10000
    assert _lib.bst_device_count() >= 0
    assert _lib.bst_tune_get(99) == -1


def test_tuning_keys_validated(built_lib):
    """Tuning values are host state: the batch stream count is checked on set."""
    from paper_2209_00220_amd import _lib

    saved = _lib.bst_tune_get(_lib.TUNE_BATCH_STREAMS)
    assert saved == 1
    for bad in (0, 5, -1):
        with pytest.raises(RuntimeError):
            _lib.bst_tune_set(_lib.TUNE_BATCH_STREAMS, bad)
    assert _lib.bst_tune_get(_lib.TUNE_BATCH_STREAMS) == saved
    _lib.bst_tune_set(_lib.TUNE_BATCH_STREAMS, 3)
    assert _lib.bst_tune_get(_lib.TUNE_BATCH_STREAMS) == 3
    _lib.bst_tune_set(_lib.TUNE_BATCH_STREAMS, saved)


def test_solo_threshold_validated(built_lib):
    from paper_2209_00220_amd import _lib

    saved = _lib.bst_tune_get(_lib.TUNE_BATCH_SOLO_TILES)
    assert saved == 16384
    with pytest.raises(RuntimeError):
        _lib.bst_tune_set(_lib.TUNE_BATCH_SOLO_TILES, 0)
    assert _lib.bst_tune_get(_lib.TUNE_BATCH_SOLO_TILES) == saved


def test_upload_rejects_misaligned_buffers(built_lib):
    """bst_upload checks every used device buffer for 16-byte alignment before it
    copies anything (so this runs without a GPU: no HIP call is reached)."""
    import numpy as np

    from paper_2209_00220_amd import _lib
    from paper_2209_00220_amd.column import HostColumn

    hc = HostColumn.from_values(np.arange(5000, dtype=np.uint32) % 300, "ppvbs")
    try:
        used = [s for s in range(_lib.NBUF) if hc.info.bytes[s]]
        assert used
        ptrs = [0] * _lib.NBUF
        ptrs[used[0]] = 0x10008   # 8-byte aligned only
        with pytest.raises(RuntimeError, match="16-byte aligned"):
            _lib.bst_upload(hc.h, ptrs, 0)
    finally:
        hc.close()


def test_probe_arguments_checked_before_any_launch(built_lib):
    """The streaming probe validates its arguments on the host (no GPU needed)."""
    from paper_2209_00220_amd import _lib

    with pytest.raises(RuntimeError, match="NULL"):
        _lib.bst_stream_probe(0, 2048, 0x10000, 0)
    with pytest.raises(RuntimeError, match="multiple of 2048"):
        _lib.bst_stream_probe(0x10000, 1000, 0x20000, 0)
    with pytest.raises(RuntimeError, match="aligned"):
        _lib.bst_stream_probe(0x10008, 2048, 0x20000, 0)
