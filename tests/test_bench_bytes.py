"""The byte counts behind the 3-D roofline figures of bench.py, recounted
independently: each pass of the face-lattice convolution as (elements
loaded, elements stored) per array, from its launch shape (lines or
column tiles, nload, nstore), summed over the arrays it runs on."""
import bench


def _tally(na, nb, nc, Pa, Pb, Pc, ns):
    passes = [
        # (arrays, lines or columns, elements loaded per line, stored per line)
        (2 * ns, na * nb, nc, Pc),          # lines along c from the compact strengths
        (2 * ns, na * Pc, nb, Pb),          # columns along b, planes a < na
    ]
    total = sum(arr * n * (ld + st) for arr, n, ld, st in passes)
    # fused normal-axis pass per set: both kinds' na rows in, kind 0's na
    # rows out, and the stored octant [Pa/2+1][Pb/2+1][Pc/2+1] of each of the
    # two kernel spectra (the kernels read the mirrored entry of that octant)
    octant = (Pa // 2 + 1) * (Pb // 2 + 1) * (Pc // 2 + 1)
    total += ns * (Pb * Pc * (2 * na + na) + 2 * octant)
    total += ns * (na * Pc * (Pb + nb))      # inverse columns along b, kind 0
    total += ns * (na * nb * (Pc + nc))      # inverse lines along c into the compact field
    return 8 * total


def test_pass_bytes_match_an_independent_tally():
    for shape in [(33, 128, 128, 72, 256, 256, 3), (4, 9, 7, 8, 18, 15, 2), (1, 5, 3, 1, 9, 5, 1)]:
        assert bench.conv3d_pass_bytes(*shape) == _tally(*shape)


def test_textbook_count_and_ordering():
    Pa, Pb, Pc, ns = 72, 256, 256, 3
    P = Pa * Pb * Pc
    assert bench.conv3d_textbook_bytes(Pa, Pb, Pc, ns) == 8 * ns * 20 * P
    assert bench.conv3d_pass_bytes(33, 128, 128, Pa, Pb, Pc, ns) < bench.conv3d_textbook_bytes(Pa, Pb, Pc, ns)


def test_sphere_lattice_pass_bytes_value():
    """At the sphere workload's lattice (3 sets of 33 x 128 x 128 padded to
    72 x 256 x 256) the passes move 535.6 MB, of which the octant spectra
    are 29.6 MB."""
    b = bench.conv3d_pass_bytes(33, 128, 128, 72, 256, 256, 3)
    assert b == 535_623_408, b
    assert 3 * 2 * 37 * 129 * 129 * 8 == 29_554_416
