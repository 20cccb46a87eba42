"""The seeded input generators against their published definitions and against the
recipes they implement (CPU only).  These fields stand in for the paper's images and
SPE10 slices, so what is pinned here is the structure each recipe promises: value
range, contrast, channels that cross the domain, layers."""
from collections import deque

import numpy as np
import pytest

from paper_1602_04858_amd import inputs


def test_splitmix64_published_sequence():
    # reference outputs of SplitMix64 (Steele, Lea, Flood 2014; Vigna's C code) for
    # the seeds 1234567 and 0
    assert [int(v) for v in inputs.splitmix64(1234567, 5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431, 16408922859458223821]
    assert [int(v) for v in inputs.splitmix64(0, 3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # offsets continue the same stream
    assert np.array_equal(inputs.splitmix64(99, 4, 6), inputs.splitmix64(99, 10)[6:])


def test_uniform_and_box_muller():
    u = inputs.uniform(7, 200000)
    assert u.min() > 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 5e-3
    z = inputs.normal(7, 200000)
    assert abs(z.mean()) < 1e-2 and abs(z.std() - 1.0) < 1e-2
    # Box-Muller by definition: a pair (z0, z1) from (u1, u2) has z0^2 + z1^2 = -2 ln u1
    # and angle 2 pi u2
    u1, u2 = inputs.uniform(7, 2)
    assert abs(z[0] ** 2 + z[1] ** 2 + 2.0 * np.log(u1)) < 1e-12
    assert abs(np.arctan2(z[1], z[0]) % (2 * np.pi) - 2 * np.pi * u2) < 1e-12


def _crosses(mask, axis):
    """A 4-connected path of True cells from one side of the grid to the other
    (axis 1: from column 0 to column n-1; axis 0: from row 0 to row n-1)."""
    n = mask.shape[0]
    seen = np.zeros_like(mask)
    q = deque()
    for i in range(n):
        a, b = (i, 0) if axis == 1 else (0, i)
        if mask[a, b]:
            seen[a, b] = True
            q.append((a, b))
    while q:
        a, b = q.popleft()
        if (b if axis == 1 else a) == n - 1:
            return True
        for da, db in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            x, y = a + da, b + db
            if 0 <= x < n and 0 <= y < n and mask[x, y] and not seen[x, y]:
                seen[x, y] = True
                q.append((x, y))
    return False


def test_lognormal_channel_field_recipe():
    n = 128
    g = np.log10(inputs.kappa_lognormal_channels(n, 2000)).reshape(n, n)
    assert g.min() >= -6.0 - 1e-12 and g.max() <= 1e-12
    top = np.isclose(g, 0.0)
    # 20 channels two cells wide and n long (overlaps aside) plus the ~2% of cells
    # whose normal draw is clipped at the top
    assert 0.15 < top.mean() < 0.7
    # channels run from side to side in both directions
    assert _crosses(top, 1) and _crosses(top, 0)
    inner = g[(g > -6.0) & (g < 0.0)]
    assert abs(inner.mean() + 3.0) < 0.15 and 1.1 < inner.std() < 1.5
    # contrast 1e6 is reached
    assert g.max() - g.min() > 5.9


def test_layered_field_recipe():
    n, layers = 170, 85
    g = np.log10(inputs.kappa_layered(n, 5000, layers=layers)).reshape(n, n)
    assert g.min() >= -6.0 - 1e-12 and g.max() <= 1.0 + 1e-12
    top = np.isclose(g, 1.0)
    assert _crosses(top, 1) or _crosses(top, 0)
    # each layer (two rows here) has its own mean, drawn from U[-5, 0]: the spread of
    # the row-band medians (channel and top-clipped cells left out) is that of the
    # layer means (variance 25/12), far above the spread inside a band (variance ~1)
    band = []
    for l in range(layers):
        rows = g[(l * n) // layers:((l + 1) * n) // layers]
        cells = rows[rows < 1.0]
        if cells.size >= n // 2:
            band.append(np.median(cells))
    band = np.array(band)
    assert band.size > layers // 2
    assert 1.0 < band.var() < 3.5 and band.min() > -6.0 and band.max() < 1.0


def test_layered3_field_recipe():
    n = 32
    g = np.log10(inputs.kappa_layered3(n, 6000)).reshape(n, n, n)  # [cz, cy, cx]
    assert g.min() >= -6.0 - 1e-12 and g.max() <= 1.0 + 1e-12
    slab = np.array([np.median(g[z]) for z in range(n)])
    within = np.array([g[z].std() for z in range(n)])
    assert slab.var() > 0.5 and np.all(within < 1.2)


def test_workloads_are_deterministic_and_distinct():
    a, b = inputs.workload("C2"), inputs.workload("C2")
    assert np.array_equal(a.kappa, b.kappa)
    c0, c1 = inputs.workload("C4", 0), inputs.workload("C4", 1)
    assert c0.kappa.size != c1.kappa.size or not np.array_equal(c0.kappa, c1.kappa)


def _components(img):
    from scipy import ndimage
    lab, n = ndimage.label(img)
    return lab, n


def _spans(lab, n, axis):
    """Some component touches both edges across `axis` (1: left to right)."""
    first = set(np.unique(np.take(lab, 0, axis=axis))) - {0}
    last = set(np.unique(np.take(lab, -1, axis=axis))) - {0}
    return bool(first & last)


def test_two_phase_images_recipe():
    """Foam: Voronoi walls that span the domain both ways; inclusions: disjoint disks
    (one component per disk, about 20% of the area, none touching another); connected
    inclusions: the same disks joined so that the structure spans left to right."""
    m = 128
    foam = inputs.phase_image("foam", 7100, m)
    lab, n = _components(foam)
    assert 0.15 < foam.mean() < 0.35
    assert _spans(lab, n, 1) and _spans(lab, n, 0)
    inc = inputs.phase_image("inclusions", 7100, m)
    st = inputs._Stream(7100)
    disks = inputs._disks(st, m, 0.20, 3.0, 8.0, overlap=False)
    lab, n = _components(inc)
    assert n == len(disks) and 0.15 < inc.mean() < 0.25
    assert not _spans(lab, n, 1) and not _spans(lab, n, 0)
    con = inputs.phase_image("connected", 7100, m)
    lab, n = _components(con)
    assert np.all(con[inc])                    # the disks are kept, bands added
    assert n < len(disks) // 3 and _spans(lab, n, 1)


def test_two_phase_kappa_values_and_refinement():
    m, e = 128, 5
    img = inputs.phase_image("connected", 7200, m)
    for n in (128, 256):
        ka = inputs.kappa_two_phase("connected", 7200, n, e).reshape(n, n)
        kb = inputs.kappa_two_phase("connected", 7200, n, e, reverse=True).reshape(n, n)
        r = n // m
        assert set(np.unique(ka)) == {10.0 ** -e, 1.0}
        # every pixel covers an r x r block of cells carrying its value
        assert np.array_equal(ka[::r, ::r] == 10.0 ** -e, img)
        assert np.array_equal(ka, np.repeat(np.repeat(ka[::r, ::r], r, 0), r, 1))
        # case (b) swaps the phases
        assert np.array_equal(kb == 1.0, ka == 10.0 ** -e)
    with pytest.raises(ValueError):
        inputs.kappa_two_phase("foam", 1, 100, 4)
