"""The C ABI: exported symbols and host-side validation (no GPU needed)."""
import ctypes

import pytest

import paper_2202_13926_amd as fsr
from paper_2202_13926_amd import binding


@pytest.fixture(scope="module")
def lib():
    return fsr.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = fsr.declared_functions()
    assert "fsr_reconstruct" in names and "fsr_context_create" in names
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for code in range(8):
        assert lib.fsr_status_string(code).decode().startswith("FSR_")


def test_defaults_and_block_count(lib):
    p = fsr.fsr_params_default()
    assert (p.block, p.border, p.iterations, p.dft, p.flags) == (4, 14, 100, 0, 0)
    assert abs(p.rho - 0.7) < 1e-7 and p.gamma == 0.5
    assert fsr.fsr_num_blocks(1080, 1920, 4) == 129600
    assert fsr.fsr_num_blocks(37, 50, 4) == 10 * 13
    assert fsr.fsr_num_blocks(0, 5, 4) == -1


@pytest.mark.parametrize("kw", [
    dict(block=0), dict(border=-1), dict(block=3), dict(block=4, border=15),
    dict(iterations=-1), dict(rho=0.0), dict(rho=1.5), dict(gamma=0.0), dict(gamma=1.01),
    dict(rho=float("nan")), dict(dft=7), dict(flags=2), dict(flags=0x80000001),
])
def test_invalid_params_rejected(lib, kw):
    with pytest.raises(fsr.FsrError) as e:
        fsr.fsr_params_validate(fsr.make_params(**kw))
    assert e.value.status == binding.FSR_ERR_INVALID_ARG
    assert lib.fsr_last_error_message().decode()


def test_valid_params_accepted():
    for kw in (dict(), dict(block=2, border=15), dict(block=8, border=12, iterations=0),
               dict(rho=1.0, gamma=1.0), dict(block=4, border=6),
               dict(flags=fsr.FSR_FLAG_LDS_ARGMAX), dict(dft=fsr.FSR_DFT_SPLIT_BF16)):
        fsr.fsr_params_validate(fsr.make_params(**kw))


def _call(lib, ctx, image, mask, out, H, W, stride, params, log=None):
    return lib.fsr_reconstruct(ctx, image, mask, out, H, W, stride, ctypes.byref(params), log, None)


def test_reconstruct_validates_before_touching_the_device(lib):
    p = fsr.make_params()
    fake_ctx = ctypes.c_void_p(0x1000)        # never dereferenced: validation fails first
    img, msk, out = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000000), ctypes.c_void_p(0x40000000)
    assert _call(lib, None, img, msk, out, 8, 8, 8, p) == binding.FSR_ERR_INVALID_ARG
    assert _call(lib, fake_ctx, None, msk, out, 8, 8, 8, p) == binding.FSR_ERR_INVALID_ARG
    assert _call(lib, fake_ctx, img, msk, out, 0, 8, 8, p) == binding.FSR_ERR_INVALID_ARG
    assert _call(lib, fake_ctx, img, msk, out, 8, 8, 7, p) == binding.FSR_ERR_INVALID_ARG
    # out overlapping image
    assert _call(lib, fake_ctx, img, msk, ctypes.c_void_p(0x10000 + 64), 8, 8, 8, p) == binding.FSR_ERR_INVALID_ARG
    # out overlapping mask
    assert _call(lib, fake_ctx, img, msk, ctypes.c_void_p(0x20000000 + 8), 8, 8, 8, p) == binding.FSR_ERR_INVALID_ARG
    # valid but outside what the library runs: support 12 and 20
    for p_other in (fsr.make_params(block=4, border=4), fsr.make_params(block=4, border=8)):
        assert _call(lib, fake_ctx, img, msk, out, 8, 8, 8, p_other) == binding.FSR_ERR_UNSUPPORTED
    # the smaller supports run with the FP32 DFT only (the LDS argmax flag is
    # accepted there too)
    p16 = fsr.make_params(block=4, border=6, dft=fsr.FSR_DFT_SPLIT_BF16)
    assert _call(lib, fake_ctx, img, msk, out, 8, 8, 8, p16) == binding.FSR_ERR_UNSUPPORTED
    assert _call(lib, fake_ctx, img, msk, out, 8, 8, 8, fsr.make_params(block=12, border=10)) == binding.FSR_ERR_UNSUPPORTED
    # the LDS-argmax ablation runs with the FP32 FFTs only
    lds_bf16 = fsr.make_params(flags=fsr.FSR_FLAG_LDS_ARGMAX, dft=fsr.FSR_DFT_SPLIT_BF16)
    assert _call(lib, fake_ctx, img, msk, out, 8, 8, 8, lds_bf16) == binding.FSR_ERR_UNSUPPORTED


def test_reuse_variant_validates_before_touching_the_device(lib):
    p = fsr.make_params()
    fake_ctx = ctypes.c_void_p(0x1000)        # never dereferenced: validation fails first
    img, msk, out = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000000), ctypes.c_void_p(0x40000000)

    def call(ctx, i, m, o, H, W, stride, params, delta):
        return lib.fsr_reconstruct_reuse(ctx, i, m, o, H, W, stride, ctypes.byref(params), delta,
                                         None, None)

    assert call(None, img, msk, out, 8, 8, 8, p, 0.5) == binding.FSR_ERR_INVALID_ARG
    assert call(fake_ctx, None, msk, out, 8, 8, 8, p, 0.5) == binding.FSR_ERR_INVALID_ARG
    assert call(fake_ctx, img, msk, out, 8, 8, 7, p, 0.5) == binding.FSR_ERR_INVALID_ARG
    assert call(fake_ctx, img, msk, ctypes.c_void_p(0x10000 + 64), 8, 8, 8, p, 0.5) == binding.FSR_ERR_INVALID_ARG
    for bad in (-0.25, 1.5, float("nan")):
        assert call(fake_ctx, img, msk, out, 8, 8, 8, p, bad) == binding.FSR_ERR_INVALID_ARG
    # S = 32 with the FP32 FFTs and no flags only
    for p_other in (fsr.make_params(block=4, border=6), fsr.make_params(dft=fsr.FSR_DFT_SPLIT_BF16),
                    fsr.make_params(flags=fsr.FSR_FLAG_LDS_ARGMAX)):
        assert call(fake_ctx, img, msk, out, 8, 8, 8, p_other, 0.5) == binding.FSR_ERR_UNSUPPORTED
    assert "reuse" in lib.fsr_last_error_message().decode()

    def frames(n, H, W, stride, fstride, o=out, delta=0.5, params=p):
        return lib.fsr_reconstruct_reuse_frames(fake_ctx, img, msk, o, n, H, W, stride, fstride,
                                                ctypes.byref(params), delta, None, None)

    for n in (0, -1, 65536):
        assert frames(n, 8, 8, 8, 64) == binding.FSR_ERR_INVALID_ARG
    assert frames(2, 8, 8, 8, 63) == binding.FSR_ERR_INVALID_ARG      # frames overlap
    # the last frame of out reaches into the image's range
    assert frames(4, 8, 8, 8, 0x1000000, o=ctypes.c_void_p(0x10000 + 0x8000000)) == binding.FSR_ERR_INVALID_ARG
    assert frames(2, 8, 8, 8, 64, delta=2.0) == binding.FSR_ERR_INVALID_ARG
    assert frames(2, 8, 8, 8, 64, params=fsr.make_params(block=4, border=6)) == binding.FSR_ERR_UNSUPPORTED


def test_tuning_import_rejects_malformed_text_before_touching_the_context(lib):
    fake_ctx = ctypes.c_void_p(0x1000)        # never dereferenced: parsing fails first
    good_head = '{"format": "fsr-batch-tuning-1", "arch": "gfx950", "cus": 256, "entries": '
    bad = ["", "{}", "[", good_head + "[]", good_head + "[[1, 3, 0, 10]]}",     # waves 3
           good_head + "[[1, 1, 65, 10]]}", good_head + "[[1, 1, 4, 33]]}",     # chunk, groups
           good_head + "[[1, 1, 0]]}", good_head + "[]} x",
           '{"format": "other", "arch": "gfx950", "cus": 256, "entries": []}',
           '{"format": "fsr-batch-tuning-1", "arch": "gfx\\950", "cus": 256, "entries": []}',
           '{"format": "fsr-batch-tuning-1", "cus": 256, "entries": []}',
           '{"format": "fsr-batch-tuning-1", "arch": "gfx950", "cus": 256, "entries": [], "x": 1}']
    for text in bad:
        assert lib.fsr_batch_tuning_import(fake_ctx, text.encode()) == binding.FSR_ERR_INVALID_ARG, text
    assert lib.fsr_batch_tuning_import(None, b"{}") == binding.FSR_ERR_INVALID_ARG
    assert lib.fsr_batch_tuning_import(fake_ctx, None) == binding.FSR_ERR_INVALID_ARG
    n = ctypes.c_size_t(0)
    assert lib.fsr_batch_tuning_export(None, None, 0, ctypes.byref(n)) == binding.FSR_ERR_INVALID_ARG


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(fsr.FsrError):
        binding.load_library(str(tmp_path / "nope.so"))


def test_batched_workspace_size(lib):
    assert fsr.fsr_batched_workspace_size(0) == 256
    assert fsr.fsr_batched_workspace_size(1) == 512
    assert fsr.fsr_batched_workspace_size(64) == 256 + 64 * 64
    with pytest.raises(fsr.FsrError):
        fsr.fsr_batched_workspace_size(-1)


def test_batched_validates_before_touching_the_device(lib):
    p = fsr.make_params()
    ctx = ctypes.c_void_p(0x1000)            # never dereferenced: validation fails first
    good = binding.fsr_image_desc(0x10000, 0x20000000, 0x40000000, None, 8, 8, 8, 10, 0)

    def call(descs, n, ws=0x50000000, ws_bytes=1 << 20, sched=None, params=p):
        arr = (binding.fsr_image_desc * max(n, 1))(*descs) if descs is not None else None
        return lib.fsr_reconstruct_batched(ctx, arr, n, ctypes.byref(params),
                                           ctypes.byref(sched) if sched else None,
                                           ws, ws_bytes, None)

    E = binding.FSR_ERR_INVALID_ARG
    assert call([good], -1) == E
    assert call(None, 2) == E
    bad = binding.fsr_image_desc(0x10000, 0x20000000, 0x40000000, None, 8, 8, 8, 10, 1)
    assert call([good, bad], 2) == E                                   # reserved != 0
    neg = binding.fsr_image_desc(0x10000, 0x20000000, 0x40000000, None, 8, 8, 8, -1, 0)
    assert call([neg], 1) == E                                         # iterations < 0
    alias = binding.fsr_image_desc(0x10000, 0x20000000, 0x10000 + 4, None, 8, 8, 8, 10, 0)
    assert call([alias], 1) == E                                       # out overlaps image
    assert call([good], 1, ws_bytes=100) == E                          # workspace too small
    assert call([good], 1, ws=None) == E
    for s in (fsr.make_schedule(3, 0, 10), fsr.make_schedule(1, 65, 10), fsr.make_schedule(1, 4, 0), fsr.make_schedule(1, 4, 33),
              binding.fsr_batch_schedule(1, 0, 10, 7)):
        assert call([good], 1, sched=s) == E
    assert call([good], 1, params=fsr.make_params(block=4, border=4)) == binding.FSR_ERR_UNSUPPORTED
    assert call([good], 1, params=fsr.make_params(block=4, border=6, dft=fsr.FSR_DFT_SPLIT_BF16)) == \
        binding.FSR_ERR_UNSUPPORTED
    assert call([good], 1, params=fsr.make_params(flags=fsr.FSR_FLAG_LDS_ARGMAX)) == binding.FSR_ERR_UNSUPPORTED
    assert lib.fsr_last_error_message().decode()
    out = ctypes.c_void_p()
    arr = (binding.fsr_image_desc * 1)(good)
    assert lib.fsr_batch_graph_create(ctx, arr, 1, ctypes.byref(p), None, None, 1 << 20,
                                      ctypes.byref(out)) == E
    assert lib.fsr_batch_graph_launch(None, None) == E
    assert lib.fsr_batch_graph_destroy(None) == binding.FSR_OK


def test_server_config_validated_before_touching_the_device(lib):
    p = fsr.make_params()
    out = ctypes.c_void_p()
    fake_ctx = ctypes.c_void_p(0x1000)       # never dereferenced: validation fails first
    E = binding.FSR_ERR_INVALID_ARG
    bad = [binding.make_server_config(hbm_budget=100), binding.make_server_config(max_inflight=0),
           binding.make_server_config(max_inflight=8, max_batch=9), binding.make_server_config(streams=3),
           binding.make_server_config(mode=5)]
    cfg = binding.make_server_config()
    cfg.reserved[2] = 1
    bad.append(cfg)
    for c in bad:
        assert lib.fsr_server_create(fake_ctx, ctypes.byref(p), ctypes.byref(c), ctypes.byref(out)) == E
    c = binding.make_server_config()
    assert lib.fsr_server_create(None, ctypes.byref(p), ctypes.byref(c), ctypes.byref(out)) == E
    for other in (fsr.make_params(block=4, border=4), fsr.make_params(block=4, border=6, dft=fsr.FSR_DFT_SPLIT_BF16)):
        assert lib.fsr_server_create(fake_ctx, ctypes.byref(other), ctypes.byref(c),
                                     ctypes.byref(out)) == binding.FSR_ERR_UNSUPPORTED
    assert lib.fsr_server_create(fake_ctx, ctypes.byref(fsr.make_params(flags=fsr.FSR_FLAG_LDS_ARGMAX)),
                                 ctypes.byref(c), ctypes.byref(out)) == binding.FSR_ERR_UNSUPPORTED
    t = ctypes.c_uint64()
    req = binding.fsr_request(0x1000, 0x2000, 8, 8, 8, 10, 0)
    assert lib.fsr_server_submit(None, ctypes.byref(req), ctypes.byref(t)) == E
    assert lib.fsr_server_destroy(None) == binding.FSR_OK
