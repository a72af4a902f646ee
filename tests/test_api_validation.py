"""The torch wrappers' argument checks, on the CPU.  Every shape, dtype and layout check
runs before the device check, so wrongly shaped CPU tensors are refused with the shape
error (on the GPU the same checks stand between the caller and the C ABI, which cannot
see tensor sizes: a wrongly sized output would be written past its end).  No call reaches
the library here."""
import pytest
import torch

from paper_1010_2641_amd import api


def z(*shape, dtype=torch.float32):
    return torch.zeros(shape, dtype=dtype)


def test_forward_out_is_checked():
    x, S = z(5, 3), z(7, 3)
    with pytest.raises(ValueError, match=r"out must have shape \(7,\)"):
        api.scatter_fwd(x, None, S, out=z(6, dtype=torch.complex64))
    with pytest.raises(ValueError, match="out must have shape"):
        api.scatter_fwd(x, None, S, out=z(7, 1, dtype=torch.complex64))
    with pytest.raises(TypeError, match="out must be torch.complex64"):
        api.scatter_fwd(x, None, S, out=z(7, dtype=torch.complex128))
    with pytest.raises(ValueError, match="out must be contiguous"):
        api.scatter_fwd(x, None, S, out=z(14, dtype=torch.complex64)[::2])
    # a well-formed call on CPU tensors reaches the device check and stops there
    with pytest.raises(ValueError, match="must be on the GPU"):
        api.scatter_fwd(x, None, S, out=z(7, dtype=torch.complex64))


def test_input_shapes_and_dtypes():
    x, S = z(5, 3), z(7, 3)
    with pytest.raises(ValueError, match="xyz must have shape"):
        api.scatter_fwd(z(5, 4), None, S)
    with pytest.raises(ValueError, match="S must have shape"):
        api.scatter_fwd(x, None, z(7))
    with pytest.raises(ValueError, match=r"f must have shape \(5,\)"):
        api.scatter_fwd(x, z(4, dtype=torch.complex64), S)
    with pytest.raises(TypeError, match="f must be torch.complex64"):
        api.scatter_fwd(x, z(5, dtype=torch.complex128), S)
    with pytest.raises(ValueError, match=r"G must have shape \(7,\)"):
        api.scatter_bwd(x, None, S, z(8, dtype=torch.complex64))
    with pytest.raises(TypeError, match="xyz must be torch.float64"):
        api.scatter_fwd_f64(x, None, S.double())
    with pytest.raises(ValueError, match=r"I must have shape \(7,\)"):
        api.loss_grad(z(7, dtype=torch.complex64), z(6))


def test_species_arrays_are_checked():
    x, S = z(4, 3), z(6, 3)
    G = z(6, dtype=torch.complex64)
    with pytest.raises(ValueError, match=r"A_species must have shape \(2, 6\)"):
        api.scatter_bwd_species(x, [0, 2, 4], None, S, G, z(3, 6, dtype=torch.complex64))
    with pytest.raises(ValueError, match=r"A_species must have shape \(2, 6\)"):
        api.scatter_bwd_species(x, [0, 2, 4], None, S, G, z(2, 5, dtype=torch.complex64))
    with pytest.raises(TypeError, match="A_species must be torch.complex64"):
        api.scatter_bwd_species(x, [0, 2, 4], None, S, G, z(2, 6))
    with pytest.raises(ValueError, match=r"fs must have shape \(2, 6\)"):
        api.scatter_bwd_species(x, [0, 2, 4], z(2, 5, dtype=torch.complex64), S, G)
    with pytest.raises(ValueError, match="must be on the GPU"):
        api.scatter_bwd_species(x, [0, 2, 4], None, S, G, z(2, 6, dtype=torch.complex64))


def test_conjugate_views():
    g = torch.tensor([1 + 2j, -3 + 0.5j], dtype=torch.complex64)
    lazy = g.conj()
    assert lazy.is_conj()
    # a lazy conjugate is refused as an input ...
    with pytest.raises(ValueError, match="conjugate view"):
        api._need(lazy, "G", torch.complex64, (2,))
    # ... and backward's seed is resolved before it is marshalled
    for dtype in (torch.complex64, torch.complex128):
        seed = api._seed_arg(lazy, dtype)
        assert not seed.is_conj() and seed.is_contiguous() and seed.dtype == dtype
        assert torch.equal(torch.view_as_real(seed),
                           torch.view_as_real(g.to(dtype)) * torch.tensor([1.0, -1.0], dtype=seed.real.dtype))


def test_grid_wrappers_are_checked():
    """The grid calls: the grid's fields and counts, the sizes of G, I and out against
    n1 n2 n3, the refusal of a factor gradient over a grid."""
    g = api.Grid((0.0, 0.0, 4.0), (0.01, 0.0, 0.0), (0.0, 0.01, 0.0), (0.0, 0.0, 0.01), 64, 2, 3)
    x = z(5, 3)
    with pytest.raises(TypeError, match="grid must be a Grid"):
        api.scatter_fwd_grid(x, None, object())
    with pytest.raises(ValueError, match="3 components"):
        api.scatter_fwd_grid(x, None, api.Grid((0.0, 0.0), (0.01, 0.0, 0.0), (0.0, 0.01, 0.0),
                                               (0.0, 0.0, 0.01), 64))
    with pytest.raises(ValueError, match="counts must be >= 0"):
        api.scatter_fwd_grid(x, None, api.Grid((0.0,) * 3, (0.01, 0.0, 0.0), (0.0,) * 3, (0.0,) * 3, -1))
    with pytest.raises(ValueError, match=r"out must have shape \(384,\)"):
        api.scatter_fwd_grid(x, None, g, out=z(383, dtype=torch.complex64))
    with pytest.raises(ValueError, match=r"G must have shape \(384,\)"):
        api.scatter_bwd_grid(x, None, g, z(100, dtype=torch.complex64))
    with pytest.raises(ValueError, match=r"I must have shape \(384,\)"):
        api.fit_step_grid(x, None, g, z(100))
    with pytest.raises(ValueError, match="must be on the GPU"):
        api.scatter_fwd_grid(x, None, g)
    f = torch.zeros(5, dtype=torch.complex64, requires_grad=True)
    with pytest.raises(NotImplementedError, match="no gradient with respect to f"):
        api.scatter_grid(x, f, g)
    assert g.size == 384


def test_species_grid_wrappers_are_checked():
    """The species-factorised calls over a grid: the partition, the factor table, the seed
    and the per-species sums against n_species x (n1 n2 n3)."""
    g = api.Grid((0.0, 0.0, 4.0), (0.01, 0.0, 0.0), (0.0, 0.01, 0.0), (0.0, 0.0, 0.01), 64, 2, 3)
    x = z(5, 3)
    with pytest.raises(ValueError, match="species_start"):
        api.scatter_fwd_species_grid(x, [0, 4], None, g)
    with pytest.raises(ValueError, match=r"fs must have shape \(2, 384\)"):
        api.scatter_fwd_species_grid(x, [0, 2, 5], z(2, 383, dtype=torch.complex64), g)
    with pytest.raises(TypeError, match="grid must be a Grid"):
        api.scatter_fwd_species_grid(x, [0, 5], None, object())
    with pytest.raises(ValueError, match=r"G must have shape \(384,\)"):
        api.scatter_bwd_species_grid(x, [0, 5], None, g, z(100, dtype=torch.complex64))
    with pytest.raises(ValueError, match=r"A_species must have shape \(2, 384\)"):
        api.scatter_bwd_species_grid(x, [0, 2, 5], None, g, z(384, dtype=torch.complex64),
                                     z(1, 384, dtype=torch.complex64))
    with pytest.raises(ValueError, match="must be on the GPU"):
        api.scatter_fwd_species_grid(x, [0, 2, 5], z(2, 384, dtype=torch.complex64), g)
    with pytest.raises(ValueError, match="must be on the GPU"):
        api.scatter_bwd_species_grid(x, [0, 5], None, g, z(384, dtype=torch.complex64))
