"""The C ABI library loads, exports every symbol include/proots.h declares,
and rejects bad arguments on the host before touching the GPU (CPU only:
no call here launches a kernel)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "proots.h")
LIB = os.path.join(ROOT, "paper_2507_02164_amd", "libproots.so")


def _ensure_built():
    if not os.path.exists(LIB):
        from paper_2507_02164_amd import build
        build.build()


@pytest.fixture(scope="module")
def lib():
    _ensure_built()
    import paper_2507_02164_amd as pr
    return pr.lib()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_three_calls():
    names = _declared_functions()
    for f in ("pr_solve", "pr_density", "pr_backward", "pr_strerror", "pr_version"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_header_and_library_serve_a_plain_c_program(lib, tmp_path):
    """tests/capi/example.c compiles as C11 with every warning an error and
    links against libproots.so: the header is valid C and declares what the
    library exports."""
    import subprocess
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    out = tmp_path / "capi_example"
    subprocess.run(["gcc", "-std=c11", "-O1", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "capi", "example.c"), "-o", str(out),
                    "-L", os.path.join(ROOT, "paper_2507_02164_amd"), "-lproots",
                    "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm"], check=True)
    assert out.exists()


def test_build_records_kernel_instruction_digests(lib):
    """The build writes a digest of every solve kernel's instructions; the
    parser keeps instruction lines only (labels, directives and comments do
    not change a digest)."""
    import json
    from paper_2507_02164_amd import build as b
    d = json.load(open(b.ISA_DIGESTS))
    timed = "_ZN6proots12_GLOBAL__N_117solve_flat_kernelILb1ELi6ELi2ELb0EEEvNS0_6PolyIOE"
    assert timed in d and len(d[timed]) == 64
    asm = "_Zk:\n  v_add_f32 v0, v1, v2 ; c\n.LBB0_1:\n  .p2align 2\n  s_endpgm\n"
    asm2 = "_Zk: ; other comment\n  v_add_f32 v0, v1, v2\n.LBB9_9:\n  s_endpgm ; end\n"
    assert b.isa_digests(asm) == b.isa_digests(asm2)
    assert b.isa_digests(asm) != b.isa_digests(asm.replace("v2", "v3"))


def test_strerror_and_version(lib):
    import paper_2507_02164_amd as pr
    assert pr.strerror(0) == "success"
    assert "invalid" in pr.strerror(-1)
    assert pr.strerror(12345) == "unknown error code"
    assert pr.version() >= 100


def test_solve_argument_validation(lib):
    import paper_2507_02164_amd as pr
    P = ctypes.c_void_p
    fake = P(0x1000)  # never dereferenced: validation fails first
    opts = pr.SolveOpts()
    assert lib.pr_solve(None, None, 10, 6, fake, fake, None, None) == pr.PR_ERR_INVALID_ARG
    assert lib.pr_solve(fake, None, -1, 6, fake, fake, None, None) == pr.PR_ERR_INVALID_ARG
    assert lib.pr_solve(fake, None, 10, 0, fake, fake, None, None) == pr.PR_ERR_INVALID_ARG
    assert lib.pr_solve(fake, None, 10, 7, fake, fake, None, None) == pr.PR_ERR_INVALID_ARG
    assert lib.pr_solve(fake, None, 10, 6, None, fake, None, None) == pr.PR_ERR_INVALID_ARG
    assert lib.pr_solve(fake, None, 10, 6, fake, None, None, None) == pr.PR_ERR_INVALID_ARG
    bad = pr.SolveOpts(precision=5)
    assert lib.pr_solve(fake, None, 10, 6, fake, fake, ctypes.byref(bad), None) == pr.PR_ERR_UNSUPPORTED
    bad = pr.SolveOpts(max_iter_per_level=-3)
    assert lib.pr_solve(fake, None, 10, 6, fake, fake, ctypes.byref(bad), None) == pr.PR_ERR_INVALID_ARG
    bad = pr.SolveOpts(polish_steps=9)
    assert lib.pr_solve(fake, None, 10, 6, fake, fake, ctypes.byref(bad), None) == pr.PR_ERR_INVALID_ARG
    bad = pr.SolveOpts(polish_tol=2.0)
    assert lib.pr_solve(fake, None, 10, 6, fake, fake, ctypes.byref(bad), None) == pr.PR_ERR_INVALID_ARG
    bad = pr.SolveOpts(flags=0x80)
    assert lib.pr_solve(fake, None, 10, 6, fake, fake, ctypes.byref(bad), None) == pr.PR_ERR_UNSUPPORTED
    bad = pr.SolveOpts(flags=0x40)
    assert lib.pr_solve(fake, None, 10, 6, fake, fake, ctypes.byref(bad), None) == pr.PR_ERR_UNSUPPORTED
    fb = pr.SolveOpts(precision=pr.FP32_POLISH, flags=pr.FLAG_FP64_FALLBACK | pr.FLAG_FIXED_STEPS |
                      pr.FLAG_RAYLEIGH_SHIFT | pr.FLAG_PAIRED_LANES | pr.FLAG_RUN_AHEAD)
    assert lib.pr_solve(fake, None, 0, 6, fake, fake, ctypes.byref(fb), None) == pr.PR_OK
    # more polynomials than one launch's grid can cover
    assert lib.pr_solve(fake, None, 0x7fffffff * 64 + 1, 6, fake, fake, None, None) == pr.PR_ERR_INVALID_ARG
    # n == 0 is a valid no-op: nothing is enqueued, the arrays may be NULL
    assert lib.pr_solve(fake, None, 0, 6, fake, fake, ctypes.byref(opts), None) == pr.PR_OK
    assert lib.pr_solve(None, None, 0, 6, None, None, None, None) == pr.PR_OK


def test_density_argument_validation(lib):
    import paper_2507_02164_amd as pr
    fake = ctypes.c_void_p(0x1000)
    ok = dict(x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, w=8, h=8)

    def call(roots=fake, hist=fake, n=4, dmax=6, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, w=8, h=8):
        return lib.pr_density(roots, None, None, 0, n, dmax, x0, x1, y0, y1, w, h, hist, None)

    assert call(roots=None) == pr.PR_ERR_INVALID_ARG
    assert call(hist=None) == pr.PR_ERR_INVALID_ARG
    assert call(n=-1) == pr.PR_ERR_INVALID_ARG
    assert call(dmax=7) == pr.PR_ERR_INVALID_ARG
    assert call(x1=-1.0) == pr.PR_ERR_INVALID_ARG
    assert call(y1=-2.0) == pr.PR_ERR_INVALID_ARG
    assert call(w=0) == pr.PR_ERR_INVALID_ARG
    assert call(h=-5) == pr.PR_ERR_INVALID_ARG
    assert call(x0=float("nan")) == pr.PR_ERR_INVALID_ARG
    assert call(x1=float("inf")) == pr.PR_ERR_INVALID_ARG
    assert call(w=65536, h=65536) == pr.PR_ERR_INVALID_ARG
    assert call(n=0) == pr.PR_OK
    assert call(n=0, roots=None) == pr.PR_OK


def test_solve_bin_argument_validation(lib):
    import paper_2507_02164_amd as pr
    f = ctypes.c_void_p(0x1000)

    def call(coeffs=f, roots=f, status=f, hist=f, n=4, dmax=6, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0,
             w=8, h=8, opts=None):
        return lib.pr_solve_bin(coeffs, None, n, dmax, roots, status, opts, 0, x0, x1, y0, y1, w,
                                h, hist, None)

    assert call(coeffs=None) == pr.PR_ERR_INVALID_ARG
    assert call(status=None) == pr.PR_ERR_INVALID_ARG
    assert call(hist=None) == pr.PR_ERR_INVALID_ARG
    assert call(n=-1) == pr.PR_ERR_INVALID_ARG
    assert call(dmax=0) == pr.PR_ERR_INVALID_ARG
    assert call(x1=-3.0) == pr.PR_ERR_INVALID_ARG
    assert call(w=0) == pr.PR_ERR_INVALID_ARG
    assert call(y0=float("nan")) == pr.PR_ERR_INVALID_ARG
    assert call(opts=ctypes.byref(pr.SolveOpts(precision=9))) == pr.PR_ERR_UNSUPPORTED
    assert call(opts=ctypes.byref(pr.SolveOpts(polish_steps=20))) == pr.PR_ERR_INVALID_ARG
    # roots may be NULL (counted, not stored); n == 0 is a no-op
    assert call(n=0, roots=None) == pr.PR_OK
    assert call(n=0, coeffs=None, roots=None, status=None) == pr.PR_OK


def test_backward_argument_validation(lib):
    import paper_2507_02164_amd as pr
    f = ctypes.c_void_p(0x1000)
    assert lib.pr_backward(None, None, f, f, 4, 6, f, f, None) == pr.PR_ERR_INVALID_ARG
    assert lib.pr_backward(f, None, None, f, 4, 6, f, f, None) == pr.PR_ERR_INVALID_ARG
    assert lib.pr_backward(f, None, f, None, 4, 6, f, f, None) == pr.PR_ERR_INVALID_ARG
    assert lib.pr_backward(f, None, f, f, 4, 6, None, f, None) == pr.PR_ERR_INVALID_ARG
    assert lib.pr_backward(f, None, f, f, 4, 6, f, None, None) == pr.PR_ERR_INVALID_ARG
    assert lib.pr_backward(f, None, f, f, -4, 6, f, f, None) == pr.PR_ERR_INVALID_ARG
    assert lib.pr_backward(f, None, f, f, 4, 0, f, f, None) == pr.PR_ERR_INVALID_ARG
    assert lib.pr_backward(f, None, f, f, 0, 6, f, f, None) == pr.PR_OK
    assert lib.pr_backward(None, None, None, None, 0, 6, None, None, None) == pr.PR_OK


def test_python_binding_refuses_cpu_tensors(lib):
    import torch
    import paper_2507_02164_amd as pr
    c = torch.zeros((7, 4), dtype=torch.complex128)
    with pytest.raises(ValueError, match="GPU"):
        pr.solve(c)
    with pytest.raises(ValueError, match="GPU"):
        pr.density(torch.zeros((6, 4), dtype=torch.complex128), (-1, 1, -1, 1), (4, 4))


def test_oracle_and_product_share_no_code():
    """The oracle tree and the HIP tree include nothing of each other."""
    import glob
    prod = glob.glob(os.path.join(ROOT, "paper_2507_02164_amd", "**", "*.*"), recursive=True)
    for f in prod:
        if f.endswith((".py", ".hip", ".hpp", ".h")):
            txt = open(f).read()
            assert "import oracle" not in txt and "from oracle" not in txt, f
            assert "oracle.c" not in txt and "liboracle" not in txt, f
    for f in glob.glob(os.path.join(ROOT, "oracle", "*.*")):
        if f.endswith((".py", ".c", ".h")):
            txt = open(f).read()
            assert "paper_2507_02164_amd" not in txt and "proots.h" not in txt, f


def test_autotune_cache_roundtrip(tmp_path, monkeypatch):
    """Cache keys and lookups (no GPU: only the JSON side)."""
    from paper_2507_02164_amd import autotune
    monkeypatch.setenv("PROOTS_TUNE_CACHE", str(tmp_path / "c.json"))
    monkeypatch.setattr(autotune, "_cache", None)
    k = autotune.key("gfx950", "fp32_polish", 6, True)
    assert k == "gfx950/fp32_polish/dmax6/mixed"
    autotune.save(k, {"options": {"tile": 1024, "grid_blocks": 2048, "max_iter_per_level": 30}})
    monkeypatch.setattr(autotune, "_cache", None)
    assert autotune.load_cache()[k]["options"]["tile"] == 1024


def test_autotune_small_batch_lookup():
    """A small uniform batch takes its own key when tuned, else the uniform
    one; mixed batches and larger ones never take it (no GPU: dict lookups)."""
    from paper_2507_02164_amd import autotune
    big = autotune.key("gfx950", "fp64", 6, False)
    small = autotune.key("gfx950", "fp64", 6, False, small=True)
    mixed = autotune.key("gfx950", "fp64", 6, True)
    assert small == "gfx950/fp64/dmax6/uniform_small" and big == "gfx950/fp64/dmax6/uniform"
    cache = {big: {"options": {"tile": -1}}, small: {"options": {"tile": -1, "ahead": 1}},
             mixed: {"options": {"tile": 1024, "ahead": 1}}}
    lim = autotune.small_limit(256)
    assert lim == 256 * 4 * 64 * autotune.SMALL_WAVES_PER_SIMD
    look = lambda mx, n, c=cache: autotune.lookup(c, "gfx950", "fp64", 6, mx, n, 256)
    assert look(False, 65536) == {"tile": -1, "ahead": 1}
    assert look(False, lim) == {"tile": -1, "ahead": 1}
    assert look(False, lim + 1) == {"tile": -1}
    assert look(False, None) == {"tile": -1}
    assert look(True, 1000) == {"tile": 1024, "ahead": 1}
    assert look(False, 1000, {big: cache[big]}) == {"tile": -1}   # small key not tuned
    assert look(False, 1000, {}) == {}


def test_committed_tuning_cache_is_valid():
    import json
    from paper_2507_02164_amd import autotune
    if not os.path.exists(autotune.DEFAULT_CACHE):
        pytest.skip("no tuning cache committed yet")
    c = json.load(open(autotune.DEFAULT_CACHE))
    for k, rec in c.items():
        o = rec["options"]
        assert -1 <= o.get("tile", 0) <= 4096
        assert o.get("grid_blocks", 0) >= 0
        assert 1 <= o.get("max_iter_per_level", 30) <= 1000


def test_density_sorted_workspace_and_argument_validation(lib):
    """Workspace sizes (a host call) and the checks pr_density_sorted makes
    before anything is enqueued."""
    import paper_2507_02164_amd as pr
    f = ctypes.c_void_p(0x1000)
    W = lib.pr_density_sorted_workspace
    assert W(-1, 6, 8, 8) == pr.PR_ERR_INVALID_ARG
    assert W(10, 0, 8, 8) == pr.PR_ERR_INVALID_ARG
    assert W(10, 7, 8, 8) == pr.PR_ERR_INVALID_ARG
    assert W(10, 6, 0, 8) == pr.PR_ERR_INVALID_ARG
    assert W(10, 6, 65536, 65536) == pr.PR_ERR_INVALID_ARG
    assert W(0, 6, 256, 256) == 0
    # beyond 2^24 pixels (or 2^31 roots) the call counts directly: no workspace
    assert W(1000, 6, 8192, 4096) == 0
    assert W(2 ** 29, 6, 256, 256) == 0
    # the sorted offsets take 2 bytes per root slot, the partial tiles 64 KiB each
    w1, w2 = W(1000, 6, 1920, 1080), W(2000, 6, 1920, 1080)
    assert w1 > 2 * 6 * 1000 and w2 - w1 >= 2 * 6 * 1000 and w1 % 256 == 0
    assert W(1 << 24, 6, 1920, 1080) >= 2 * 6 * (1 << 24) + 127 * 65536

    need = W(4, 6, 8, 8)

    def call(ws=f, nbytes=need, roots=f, hist=f, n=4, dmax=6, w=8, h=8, x1=1.0):
        return lib.pr_density_sorted(roots, None, None, 0, n, dmax, -1.0, x1, -1.0, 1.0, w, h, hist,
                                     ws, nbytes, None)

    assert call(ws=None) == pr.PR_ERR_NO_MEMORY
    assert call(nbytes=need - 1) == pr.PR_ERR_NO_MEMORY
    assert call(ws=ctypes.c_void_p(0x1010)) == pr.PR_ERR_INVALID_ARG     # not 256-aligned
    assert call(roots=None) == pr.PR_ERR_INVALID_ARG
    assert call(hist=None) == pr.PR_ERR_INVALID_ARG
    assert call(dmax=0) == pr.PR_ERR_INVALID_ARG
    assert call(x1=-2.0) == pr.PR_ERR_INVALID_ARG
    assert call(n=-1) == pr.PR_ERR_INVALID_ARG
    assert call(n=0, ws=None, nbytes=0) == pr.PR_OK
    assert pr.strerror(pr.PR_ERR_NO_MEMORY).startswith("workspace")
