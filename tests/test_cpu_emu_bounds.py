"""Memory-access check of the Cholesky and tension-solve kernels and their
launch schedules on the CPU: the sources are compiled as host C++ against a
stand-in HIP runtime
that runs every thread of every launch in turn, under AddressSanitizer, with
buffers of exactly the sizes the library documents (matrix (n-1)*ld + n
doubles, workspace bd_workspace_size bytes).  Any out-of-bounds read or
write of any kernel thread fails the run with the kernel and source line.
No GPU is used."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CLANG = "/opt/rocm/llvm/bin/clang++"


def _build(tmp_path_factory, name):
    if not os.path.exists(CLANG) and shutil.which("clang++") is None:
        pytest.skip("no clang++ for the host build")
    cxx = CLANG if os.path.exists(CLANG) else shutil.which("clang++")
    exe = str(tmp_path_factory.mktemp("emu") / name)
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-I", os.path.join(HERE, "cpu_emu"), "-I", os.path.join(ROOT, "include"),
           "-x", "c++", os.path.join(HERE, "cpu_emu", name + ".cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    return _build(tmp_path_factory, "chol_emu")


@pytest.fixture(scope="module")
def cemu(tmp_path_factory):
    return _build(tmp_path_factory, "constrain_emu")


@pytest.fixture(scope="module")
def bemu(tmp_path_factory):
    return _build(tmp_path_factory, "chol_batch_emu")


@pytest.fixture(scope="module")
def cbemu(tmp_path_factory):
    return _build(tmp_path_factory, "constrain_batch_emu")


CASES = [(n, ld_pad) for n in (1, 6, 127, 128, 129, 256, 257, 383, 640, 1101, 3003) for ld_pad in (0, 3)]


@pytest.mark.parametrize("n,ld_pad", CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_cholesky_accesses_in_bounds(emu, n, ld_pad, prec):
    # every step width (1, 2 or 4 panels, and 4 turning to 2 halfway) with
    # and without lookahead on the matrix-core diagonal-block kernel, and the
    # default schedule with the register-tiled one
    runs = [(sp, la, 1, 0) for sp in (1, 2, 4) for la in (0, 1)]
    runs += [(4, la, 1, n // 2) for la in (0, 1)] + [(4, 1, 0, n // 2)]
    for sp, la, tile, wide in runs:
        r = subprocess.run([emu, str(n), str(n + ld_pad), str(prec), str(sp), str(la), str(tile),
                            str(wide)], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, (n, ld_pad, prec, sp, la, tile, wide, r.stderr[-3000:])
        assert "status 0" in r.stdout and " 0 schedule errors" in r.stdout


# (beads, Newton iteration cap, skip the matrix-free product threads): the
# largest chain the solve supports runs with the O(N^2) product skipped.
@pytest.mark.parametrize("N,maxit,skip", [(2, 1, 0), (3, 2, 0), (37, 2, 0), (300, 1, 0),
                                          (1025, 1, 1), (4097, 2, 1), (4098, 1, 1),
                                          (8193, 2, 1)])
def test_constrain_accesses_in_bounds(cemu, N, maxit, skip):
    r = subprocess.run([cemu, str(N), str(maxit), str(skip)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, (N, maxit, skip, r.stderr[-3000:])
    assert "status 0" in r.stdout


# The one-launch solve (grid barriers, the product with two phase sets per
# wave, the controller passes) with one workgroup, whose barriers never wait.
@pytest.mark.parametrize("N,maxit", [(2, 1), (3, 2), (37, 2), (300, 1)])
def test_one_launch_constrain_accesses_in_bounds(cemu, N, maxit):
    r = subprocess.run([cemu, str(N), str(maxit), "0", "1"], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, (N, maxit, r.stderr[-3000:])
    assert "status 0" in r.stdout


# Ensembles: chains of uneven sizes (one panel or less, ragged last panels,
# exact multiples of the step) factored in shared launches, each chain in
# its own exact-size buffers; and the batched tension solve.
BATCH_SIZES = ["3", "6", "384", "129", "257", "640", "128", "255", "1101"]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("lookahead", [0, 1])
@pytest.mark.parametrize("panels", [2, 4])
def test_batched_cholesky_accesses_in_bounds(bemu, prec, lookahead, panels):
    r = subprocess.run([bemu, str(prec), str(lookahead), str(panels), *BATCH_SIZES],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (prec, lookahead, panels, r.stderr[-3000:])
    assert "status 0" in r.stdout


def test_batched_constrain_accesses_in_bounds(cbemu):
    r = subprocess.run([cbemu, "2", "2", "3", "37", "300", "17", "64"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "status 0" in r.stdout and "done 6" in r.stdout


@pytest.fixture(scope="module")
def aemu(tmp_path_factory):
    return _build(tmp_path_factory, "adjoint_emu")


# The Cholesky adjoint: ragged last blocks, exact multiples of the tile,
# several join levels, padded leading dimensions, a batch of two.
@pytest.mark.parametrize("n,ld_pad", [(1, 0), (5, 2), (64, 0), (65, 1), (127, 0), (128, 3),
                                      (129, 0), (200, 5), (321, 0)])
def test_cholesky_adjoint_accesses_in_bounds(aemu, n, ld_pad):
    r = subprocess.run([aemu, str(n), str(ld_pad)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (n, ld_pad, r.stderr[-3000:])
    assert "status 0" in r.stdout


# The adjoints of the assembly and of the noise product (differentiation):
# ragged bead counts (one tile or less, tiles with a ragged last one) and
# leading dimensions with padding.
@pytest.fixture(scope="module")
def raemu(tmp_path_factory):
    return _build(tmp_path_factory, "rpy_adjoint_emu")


@pytest.fixture(scope="module")
def baemu(tmp_path_factory):
    return _build(tmp_path_factory, "brownian_adjoint_emu")


@pytest.mark.parametrize("N,pad", [(1, 0), (2, 3), (16, 0), (17, 5), (45, 1), (130, 0)])
def test_rpy_adjoint_accesses_in_bounds(raemu, N, pad):
    r = subprocess.run([raemu, str(N), str(pad)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (N, pad, r.stderr[-3000:])
    assert "status 0 (device 0)" in r.stdout


@pytest.mark.parametrize("N,pad,padb", [(1, 0, 0), (2, 3, 0), (43, 0, 5), (86, 1, 2), (300, 0, 7)])
def test_brownian_adjoint_accesses_in_bounds(baemu, N, pad, padb):
    r = subprocess.run([baemu, str(N), str(pad), str(padb)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, (N, pad, padb, r.stderr[-3000:])
    assert "status 0" in r.stdout


# The assembly (one chain, both fills; three chains through the batched
# kernel): every element written where it belongs and nothing else, for
# bead counts that leave ragged row blocks and column bead groups and
# leading dimensions with padding.
@pytest.fixture(scope="module")
def rasemu(tmp_path_factory):
    return _build(tmp_path_factory, "rpy_emu")


@pytest.mark.parametrize("N,pad", [(1, 0), (2, 3), (5, 0), (85, 1), (86, 0), (171, 4), (300, 0), (1023, 2)])
@pytest.mark.parametrize("fill", [0, 1])
def test_rpy_assemble_accesses_in_bounds(rasemu, N, pad, fill):
    r = subprocess.run([rasemu, str(N), str(pad), str(fill)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, (N, pad, fill, r.stderr[-3000:])
    assert " 0 errors" in r.stdout
