"""A structured particle set whose binned result has a closed form, for
checks at sizes the oracle cannot bin in a test (up to 2^32 - 1 particles).

Particle i on an nx by ny mesh over [0, 1]^2 (nx, ny powers of two, so the
cell centres are exact in binary32) sits at the centre of cell
(i mod nx, (i div nx) mod ny), so its bin is i mod B with B = nx * ny.
Attribute j of particle i is ((i div B) + j) mod 3 - 1, one of -1, 0, 1.
Bin b holds the particles b + B * m for m < c_b, c_b = n div B + (b < n mod B),
and its attribute j takes the values ((m + j) mod 3) - 1 for those m, so
count, sum, min, max and average depend only on c_b and j.  The closed form
is pinned to the oracle on small sizes by a CPU test."""
import numpy as np

# The largest grids the boundary accepts (nx * ny <= 2^31 - 1), binned on the
# GPU with the sparse pattern: (n, nx, ny, binary64 coordinates).
MAX_GRID_CASES = [((1 << 26) + 77, 1 << 15, 1 << 15, False), ((1 << 26) + 77, (1 << 31) - 1, 1, True)]
MAX_GRID_IDS = ["2^15x2^15-f32", "(2^31-1)x1-f64"]


def columns(idx, nx, ny, k, xp_float):
    """Coordinates and attributes of particles idx (an integer array of
    numpy or torch); xp_float casts an integer array to binary32."""
    B = nx * ny
    x = (xp_float(idx % nx) + 0.5) / nx
    y = (xp_float((idx // nx) % ny) + 0.5) / ny
    attrs = [xp_float(((idx // B) + j) % 3 - 1) for j in range(k)]
    return x, y, attrs


def expected(n, nx, ny, k):
    """Per-bin results as the oracle returns them ([ny, nx] arrays)."""
    B = nx * ny
    q, r = divmod(n, B)
    cnt = np.full(B, q, np.int64)
    cnt[:r] += 1
    res = {"count": cnt.reshape(ny, nx), "sum": [], "min": [], "max": [], "avg": [], "abs_sum": []}
    for j in range(k):
        per = {}
        for c in {q, q + 1} if r else {q}:
            vals = [((m + j) % 3) - 1 for m in range(min(c, 3))]
            full = c // 3  # each full cycle of three values sums to 0 and has |a| sum 2
            tail = [((m + j) % 3) - 1 for m in range(3 * full, c)]
            s = float(sum(tail))
            a = float(2 * full + sum(abs(v) for v in tail))
            mn = float(min(vals)) if c else np.inf
            mx = float(max(vals)) if c else -np.inf
            per[c] = (s, mn, mx, s / c if c else np.nan, a)
        lo, hi = per[q], per.get(q + 1, per[q])
        cols = [np.where(cnt == q + 1, hi[f], lo[f]) for f in range(5)]
        for key, col in zip(("sum", "min", "max", "avg", "abs_sum"), cols):
            res[key].append(col.reshape(ny, nx))
    return res


def sparse_cells(idx, n, nx, ny):
    """Flat cell of particle i in the sparse pattern: (i * nx * ny) div n."""
    return (idx * (nx * ny)) // n


def sparse_columns(idx, n, nx, ny, k, xp_float):
    """A second pattern, spread evenly over the whole grid: particle i
    (i < n <= nx * ny) alone at the centre of flat cell (i * nx * ny) div n,
    so the used bins reach the last row of the largest grids.  Attribute j
    of particle i is (i + j) mod 3 - 1.  xp_float must hold c mod nx + 0.5
    and c div nx + 0.5 exactly (binary32 up to 2^23 cells per axis, else
    binary64)."""
    c = sparse_cells(idx, n, nx, ny)
    x = (xp_float(c % nx) + 0.5) / nx
    y = (xp_float(c // nx) + 0.5) / ny
    attrs = [xp_float((idx + j) % 3 - 1) for j in range(k)]
    return x, y, attrs


def sparse_expected(n, nx, ny, k):
    """Per-bin results of sparse_columns as the oracle returns them (small
    grids only: full [ny, nx] arrays)."""
    B = nx * ny
    idx = np.arange(n, dtype=np.int64)
    bins = sparse_cells(idx, n, nx, ny)
    cnt = np.zeros(B, np.int64)
    cnt[bins] = 1
    res = {"count": cnt.reshape(ny, nx), "sum": [], "min": [], "max": [], "avg": [], "abs_sum": []}
    for j in range(k):
        v = ((idx + j) % 3 - 1).astype(np.float64)
        for key, empty in (("sum", 0.0), ("min", np.inf), ("max", -np.inf), ("avg", np.nan), ("abs_sum", 0.0)):
            col = np.full(B, empty)
            col[bins] = np.abs(v) if key == "abs_sum" else v
            res[key].append(col.reshape(ny, nx))
    return res


def columns3(idx, nx, ny, nz, k, xp_float):
    """The lattice on an nx by ny by nz mesh (powers of two): particle i at
    the centre of cell (i mod nx, (i div nx) mod ny, (i div nx ny) mod nz),
    flat bin i mod (nx ny nz), attribute j = ((i div nx ny nz) + j) mod 3 - 1:
    the results are those of the two-axis lattice with nx * ny * nz bins."""
    B = nx * ny * nz
    x = (xp_float(idx % nx) + 0.5) / nx
    y = (xp_float((idx // nx) % ny) + 0.5) / ny
    z = (xp_float((idx // (nx * ny)) % nz) + 0.5) / nz
    attrs = [xp_float(((idx // B) + j) % 3 - 1) for j in range(k)]
    return x, y, z, attrs


def expected3(n, nx, ny, nz, k):
    """Per-bin results of columns3 shaped [nz, ny, nx]."""
    res = expected(n, nx, ny * nz, k)
    shape = (nz, ny, nx)
    return {key: (val.reshape(shape) if not isinstance(val, list) else [v.reshape(shape) for v in val])
            for key, val in res.items()}
