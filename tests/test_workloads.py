"""The input generators build what their docstrings state (geometry only: none of
the sum's arithmetic is involved)."""
import numpy as np

from paper_1010_2641_amd import workloads as wl


def test_ewald_frame_lies_on_the_sphere():
    lam, ki, kf, normal = wl.ewald_geometry((4, 0, 4))
    S = wl.ewald_scan((4, 0, 4), n_pix=(33, 17), n_frames=1)
    # k_f = S / a + k_i / lambda has length 1 / lambda for every pixel
    kf_all = S / wl.GE_A + ki[None, :] / lam
    assert np.allclose(np.linalg.norm(kf_all, axis=1) * lam, 1.0, rtol=0, atol=1e-12)
    # the centre pixel (odd sizes) sits on the node
    assert np.allclose(S[(33 * 17) // 2], [4.0, 0.0, 4.0], atol=1e-12)
    # Bragg condition of the geometry itself
    assert np.allclose((kf - ki) / lam * wl.GE_A, [4.0, 0.0, 4.0], atol=1e-12)


def test_ewald_scan_is_a_rotation_per_frame_and_not_a_grid():
    S = wl.ewald_scan((4, 0, 4), n_pix=(16, 16), n_frames=5, rock_deg=0.5)
    frames = S.reshape(5, 256, 3)
    n = np.linalg.norm(frames, axis=2)
    assert np.allclose(n, n[0][None, :], rtol=0, atol=1e-12)     # rotations keep |S|
    assert not np.allclose(frames[0], frames[-1])
    # curved sheets: no coordinate takes a few repeated values as on a product grid
    for c in range(3):
        assert len(np.unique(np.round(S[:, c], 12))) > S.shape[0] // 4


def test_cube41_matches_the_section_4_1_example():
    w = wl.cube41()
    assert w.n_atoms == 1_000_000 and w.n_points == 40_000
    assert w.xyz[:, 0].min() == -50 and w.xyz[:, 0].max() == 49 and w.xyz[:, 2].max() == 99
    assert np.isclose(w.S[:, 0].min(), -0.1) and np.isclose(w.S[:, 2].max(), 4.099)
    ws = wl.cube41(True)
    # z += 1e-6 z (x^2 + y^2): the corner atom (-50, -50, 99) moves by 0.495
    i = np.argmax(ws.xyz[:, 2])
    assert np.isclose(ws.xyz[i, 2], 99 + 1e-6 * 99 * 5000, atol=1e-4)


def test_group_by_species_is_a_stable_partition():
    rng = np.random.default_rng(3)
    f = rng.choice(np.array([1 + 1j, 2.0, 3 - 1j], dtype=np.complex64), size=50)
    xyz = rng.random((50, 3)).astype(np.float32)
    xs, start, vals, order = wl.group_by_species(xyz, f)
    assert start[0] == 0 and start[-1] == 50
    for s in range(len(vals)):
        assert np.all(f[order[start[s]:start[s + 1]]] == vals[s])
        assert np.all(np.diff(order[start[s]:start[s + 1]]) > 0)
    assert np.array_equal(xs, xyz[order])
