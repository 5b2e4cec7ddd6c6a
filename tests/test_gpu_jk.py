"""GPU parity of the FP64 J/K build against the CPU oracle (elementwise), plus
properties that hold at any size."""
import numpy as np
import pytest

import oracle
from gpu_util import blocks_of, gpu_jk, sample_pairs, say
from paper_2406_11185_amd import molgen

pytestmark = pytest.mark.gpu
TOL_ABS = 1e-10   # plain FP64 path against the FP64 oracle


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2406_11185_amd import jk as jkb
    jkb.load()


def test_w4_full_no_screening():
    mol = molgen.workload("w4")
    say("case w4 (40 functions, tol 0)")
    J, K = gpu_jk(mol, 0.0)
    Jo, Ko, _ = oracle.jk(mol, 0.0)
    say("  max|dJ| =", np.abs(J - Jo).max(), " max|dK| =", np.abs(K - Ko).max())
    assert np.abs(J - Jo).max() <= TOL_ABS
    assert np.abs(K - Ko).max() <= TOL_ABS


@pytest.mark.parametrize("nh,nH,seed,tol", [(3, 3, 21, 0.0), (4, 5, 5, 1e-8), (1, 1, 7, 0.0),
                                            (0, 3, 3, 0.0)])
def test_small_molecules_full(nh, nH, seed, tol):
    mol = molgen.make_molecule(nh, nH, seed) if nh else molgen.make_molecule(0, nH, seed,
                                                                            heavy_z=[])
    say(f"case m{nh}_{nH}_{seed} ({mol.n_bf} functions, tol {tol})")
    J, K = gpu_jk(mol, tol)
    Jo, Ko, _ = oracle.jk(mol, tol)
    say("  max|dJ| =", np.abs(J - Jo).max(), " max|dK| =", np.abs(K - Ko).max())
    assert np.abs(J - Jo).max() <= TOL_ABS
    assert np.abs(K - Ko).max() <= TOL_ABS


@pytest.mark.parametrize("nh,nH,seed,tol", [(2, 3, 5, 0.0), (3, 2, 9, 1e-8)])
def test_ragged_contraction_lengths(nh, nH, seed, tol):
    """Shells of 1, 2, 4 and 8 primitives (the library maximum): bins of 1 to 64
    primitive pairs, bra and ket bins of different lengths."""
    mol = molgen.ragged_molecule(nh, nH, seed)
    say(f"case {mol.name} ({mol.n_bf} functions, primitives {sorted(set(mol.shell_nprim.tolist()))},"
        f" tol {tol})")
    J, K = gpu_jk(mol, tol)
    Jo, Ko, _ = oracle.jk(mol, tol)
    say("  max|dJ| =", np.abs(J - Jo).max(), " max|dK| =", np.abs(K - Ko).max())
    assert np.abs(J - Jo).max() <= TOL_ABS
    assert np.abs(K - Ko).max() <= TOL_ABS


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_single_atom_boys_at_zero(precision):
    """Degenerate geometry: one atom carries every shell, so every Gaussian product
    centre coincides (A = B = P = Q) and every Boys argument is exactly 0; all
    classes, FP64 and (every quartet) FP32, against the oracle."""
    mol = molgen.make_molecule(1, 0, 13)
    say(f"case one atom ({mol.n_bf} functions, tol 0, {precision})")
    import torch
    from paper_2406_11185_amd import jk as jkb
    D = torch.as_tensor(mol.D, device="cuda")
    J, K = jkb.jk(mol, D, 0.0, precision=precision, fp32_below=1e9)
    J, K = J.cpu().numpy(), K.cpu().numpy()
    Jo, Ko, _ = oracle.jk(mol, 0.0)
    say("  max|dJ| =", np.abs(J - Jo).max(), " max|dK| =", np.abs(K - Ko).max())
    bound = TOL_ABS if precision == "fp64" else 1e-6 * max(np.abs(Jo).max(), np.abs(Ko).max())
    assert np.abs(J - Jo).max() <= bound and np.abs(K - Ko).max() <= bound


def test_multiple_densities_share_one_pass():
    mol = molgen.make_molecule(2, 2, 11, n_dm=3)
    say(f"case n_dm=3 ({mol.n_bf} functions)")
    J, K = gpu_jk(mol, 0.0)
    Jo, Ko, _ = oracle.jk(mol, 0.0)
    assert J.shape == (3, mol.n_bf, mol.n_bf)
    assert np.abs(J - Jo).max() <= TOL_ABS and np.abs(K - Ko).max() <= TOL_ABS


def test_w30_sampled_blocks():
    mol = molgen.workload("w30")
    say("case w30 (270 functions, tol 1e-10), sampled blocks")
    J, K = gpu_jk(mol, 1e-10)
    pairs = sample_pairs(mol, 9, seed=30)
    ref = oracle.jk_blocks(mol, 1e-10, pairs)
    for (m, n), gj, gk, (oj, ok) in zip(pairs, blocks_of(mol, J, pairs), blocks_of(mol, K, pairs), ref):
        say(f"  block ({m},{n}) dJ={np.abs(gj - oj).max():.2e} dK={np.abs(gk - ok).max():.2e}")
        assert np.abs(gj - oj).max() <= TOL_ABS
        assert np.abs(gk - ok).max() <= TOL_ABS
    np.testing.assert_allclose(J, J.transpose(0, 2, 1), atol=1e-13)
    np.testing.assert_allclose(K, K.transpose(0, 2, 1), atol=1e-13)


def test_w120_sampled_blocks():
    """The 1080-function molecule in FP64 at tol 1e-10, in the launch configuration
    of the benchmark's extra measurement: sampled blocks against the oracle."""
    mol = molgen.workload("w120")
    say("case w120 (1080 functions, tol 1e-10, FP64), sampled blocks")
    J, K = gpu_jk(mol, 1e-10)
    pairs = sample_pairs(mol, 4, seed=120)
    ref = oracle.jk_blocks(mol, 1e-10, pairs)
    for (m, n), gj, gk, (oj, ok) in zip(pairs, blocks_of(mol, J, pairs), blocks_of(mol, K, pairs), ref):
        say(f"  block ({m},{n}) dJ={np.abs(gj - oj).max():.2e} dK={np.abs(gk - ok).max():.2e}")
        assert np.abs(gj - oj).max() <= TOL_ABS
        assert np.abs(gk - ok).max() <= TOL_ABS


def test_w30_rank_one_identity():
    """D = c c^T, no screening: J c = K c (both equal (mu phi|phi phi))."""
    mol = molgen.workload("w30")
    say("case w30 rank-one density, tol 0")
    c = np.random.default_rng(3).normal(size=mol.n_bf) / np.sqrt(mol.n_bf)
    J, K = gpu_jk(mol, 0.0, D=np.outer(c, c)[None])
    np.testing.assert_allclose(J[0] @ c, K[0] @ c, rtol=1e-10, atol=1e-12)


def test_everything_screened():
    mol = molgen.workload("w4")
    say("case w4 tol 1e3 (every quartet screened)")
    J, K = gpu_jk(mol, 1e3)
    assert np.all(J == 0) and np.all(K == 0)


def test_argument_errors_leave_outputs_untouched():
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.workload("w4")
    say("case argument errors")
    ctx = jkb.default_context(0)
    b = jkb.Basis(mol)
    D = torch.as_tensor(mol.D, device="cuda")
    J = torch.full_like(D, 7.0)
    K = torch.full_like(D, 7.0)
    for opts, code in [(jkb.make_opts(n_dm=0), jkb.JK_EINVAL),
                       (jkb.make_opts(precision=5), jkb.JK_EINVAL),
                       (jkb.make_opts(boys_fp64_T=45.0), jkb.JK_EINVAL),
                       (jkb.make_opts(deterministic=2), jkb.JK_EINVAL),
                       (jkb.make_opts(acc_copies=9), jkb.JK_EINVAL),
                       (jkb.make_opts(serial=True, deterministic=-1), jkb.JK_EINVAL)]:
        with pytest.raises(jkb.JkError) as e:
            jkb.jk_build(ctx, b, D, J, K, 0.0, opts)
        assert e.value.code == code
    with pytest.raises(jkb.JkError):
        jkb.jk_build(ctx, b, D, J, K, -1.0, jkb.make_opts())
    torch.cuda.synchronize()
    assert torch.all(J == 7.0) and torch.all(K == 7.0)
    with pytest.raises(jkb.JkError) as e:
        jkb.jk_build(ctx, b, D, J, K, 0.0, jkb.make_opts(max_scratch_bytes=1024))
    assert e.value.code == jkb.JK_ENOMEM


def test_single_launch_build():
    """Every shell pair in one bin: the build makes a single class launch, which
    runs alone on the caller's stream with no fork to the internal streams."""
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.single_bin_molecule(7, 13)
    say(f"case single launch s7_13 ({mol.n_bf} functions, tol 0)")
    ctx = jkb.Context(0)
    D = torch.as_tensor(np.ascontiguousarray(mol.D), device="cuda")
    J, K = jkb.jk(mol, D, 0.0, timing=True, ctx=ctx)
    torch.cuda.synchronize()
    st = ctx.stats()
    assert sum(st.launches_fp64) + sum(st.launches_fp32) == 1
    Jo, Ko, _ = oracle.jk(mol, 0.0)
    dJ, dK = np.abs(J.cpu().numpy() - Jo).max(), np.abs(K.cpu().numpy() - Ko).max()
    say("  max|dJ| =", dJ, " max|dK| =", dK)
    assert dJ <= TOL_ABS and dK <= TOL_ABS
    ctx.close()
