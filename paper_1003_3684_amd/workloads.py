"""Seeded synthetic workloads (inputs only -- none of the generators' arithmetic).

Both the GPU path and the CPU oracle consume these parameter sets; neither
defines them.  The sizes and distributions follow the paper's workloads: PBA
graphs with a fixed number of edges per vertex spread over contiguous vertex
partitions (section "Parallel Barabasi-Albert (PBA) method"; Table 1 uses
1,000 processors and m = 5), and Kronecker graphs grown from a small seed or
initiator (section "Parallel Kronecker (PK) method").  The paper uses no
public dataset for generation, so nothing here stands in for one.
"""
import numpy as np

# Kronecker initiator of the 2^30-vertex workload: a 3x3 matrix zero-padded to
# 4x4 so that ids are 2-bit digit strings filling [0, 2^30).
_W3 = [[0.45, 0.20, 0.10], [0.20, 0.15, 0.05], [0.10, 0.05, 0.02]]
_W4 = [row + [0.0] for row in _W3] + [[0.0, 0.0, 0.0, 0.0]]

PBA_SMALL = dict(name="pba_n65536_m4_P64", kind="pba", n=65536, m=4, num_parts=64, p_inter=0.1, seed=1, id_bytes=4)

KRON_K20 = dict(name="kron2x2_k20_E2^24", kind="kron", n0=2, initiator=[[0.57, 0.19], [0.19, 0.05]], k=20,
                num_edges=1 << 24, seed=7, id_bytes=4)

PBA_SCALE = [dict(name=f"pba_n2^27_m5_P1024_p{p}", kind="pba", n=1 << 27, m=5, num_parts=1024, p_inter=p, seed=11,
                  id_bytes=4) for p in (0.01, 0.1, 0.3)]

KRON_SCALE = dict(name="kron3x3pad4_k15_E5x2^30", kind="kron", n0=4, initiator=_W4, k=15, num_edges=5 << 30,
                  seed=13, id_bytes=8)

KRON_SCALE_B = dict(name="kron3x3_k19_E5x2^30", kind="kron", n0=3, initiator=_W3, k=19, num_edges=5 << 30,
                    seed=13, id_bytes=8)

# Paper-scale PBA analogue of the generation-time table: 1 B vertices, m = 5.
PBA_PAPER = dict(name="pba_n2^30_m5_P1024", kind="pba", n=1 << 30, m=5, num_parts=1024, p_inter=0.1, seed=11,
                 id_bytes=4)

# Seed graph of the paper's Kronecker example (Fig. 2(b)): 5 vertices, 11 edges.
FIG2_SEED = np.array([[1, 1, 1, 1, 0],
                      [1, 1, 0, 0, 0],
                      [1, 0, 1, 0, 0],
                      [1, 0, 0, 1, 0],
                      [0, 0, 0, 0, 1]], dtype=np.uint8)


def random_kron_case(rng, max_edges=200_000):
    """A small random sample-mode Kronecker case for parity sweeps."""
    n0 = int(rng.integers(2, 5))
    k = int(rng.integers(1, 8))
    W = rng.uniform(0.0, 1.0, size=(n0, n0)).astype(np.float32)
    W[rng.uniform(size=(n0, n0)) < 0.2] = 0.0
    if W.sum() == 0:
        W[0, 0] = 1.0
    E = int(rng.integers(0, max_edges))
    return dict(n0=n0, initiator=W, k=k, num_edges=E, seed=int(rng.integers(0, 2 ** 63)), id_bytes=4)


def random_pba_case(rng, max_n=50_000):
    """A small random PBA case (default or random faction lists)."""
    P = int(rng.integers(1, 40))
    n = int(rng.integers(2 * P, max(2 * P + 1, max_n)))
    m = int(rng.integers(1, 7))
    p = float(rng.choice([0.0, 0.05, 0.1, 0.5, 1.0]))
    case = dict(n=n, m=m, num_parts=P, p_inter=p, seed=int(rng.integers(0, 2 ** 63)), id_bytes=4,
                faction_off=None, faction_members=None)
    if rng.uniform() < 0.4:
        sizes = rng.integers(1, 4, size=P)
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
        mem = rng.integers(0, P, size=int(off[-1])).astype(np.uint32)
        case["faction_off"], case["faction_members"] = off, mem
    return case


def ensemble_table(count=4096, seed=17):
    """Parameter table of a batched ensemble: graph g is PBA if g is even,
    Kronecker if odd.  PBA: n log-uniform in [2^10, 2^20], m in {2..8},
    p uniform in [0, 0.5], 64 partitions.  Kronecker: a 2x2 initiator with
    entries uniform in [0.02, 0.7], each row divided by its row sum, k
    uniform in {10..20} and 16 * 2^k edges."""
    rng = np.random.default_rng(seed)
    rows = []
    for g in range(count):
        if g % 2 == 0:
            n = int(np.floor(2.0 ** rng.uniform(10.0, 20.0)))
            rows.append(dict(kind="pba", graph_id=g, n=n, m=int(rng.integers(2, 9)),
                             p_inter=float(rng.uniform(0.0, 0.5)), num_parts=64, seed=seed))
        else:
            W = rng.uniform(0.02, 0.7, size=(2, 2)).astype(np.float32)
            W = (W / W.sum(axis=1, keepdims=True)).astype(np.float32)
            k = int(rng.integers(10, 21))
            rows.append(dict(kind="kron", graph_id=g, n0=2, initiator=W, k=k, num_edges=16 << k, seed=seed))
    return rows


def small_ensemble_table(count=48, seed=23, log2_n=(10, 14), k_range=(10, 14), parts=8):
    """The ensemble recipe at test sizes: PBA with n log-uniform in
    [2^log2_n[0], 2^log2_n[1]] and `parts` partitions; Kronecker with k in
    k_range and 16 * 2^k edges."""
    rng = np.random.default_rng(seed)
    rows = []
    for g in range(count):
        if g % 2 == 0:
            n = int(np.floor(2.0 ** rng.uniform(*log2_n)))
            rows.append(dict(kind="pba", graph_id=g, n=n, m=int(rng.integers(2, 9)),
                             p_inter=float(rng.uniform(0.0, 0.5)), num_parts=parts, seed=seed))
        else:
            W = rng.uniform(0.02, 0.7, size=(2, 2)).astype(np.float32)
            W = (W / W.sum(axis=1, keepdims=True)).astype(np.float32)
            k = int(rng.integers(k_range[0], k_range[1] + 1))
            rows.append(dict(kind="kron", graph_id=g, n0=2, initiator=W, k=k, num_edges=16 << k, seed=seed))
    return rows


def faction_groups(num_parts, groups, overlap=False):
    """Faction table of a block community topology: partition q belongs to
    group g = floor(q groups / P), whose partitions form one faction; with
    overlap, q's list also holds the next group's partitions (factions that
    share members).  Returns (faction_off, faction_members) for pba_generate."""
    members_of = [[q for q in range(num_parts) if q * groups // num_parts == g] for g in range(groups)]
    off, mem = [0], []
    for q in range(num_parts):
        g = q * groups // num_parts
        lst = list(members_of[g])
        if overlap:
            lst += members_of[(g + 1) % groups]
        mem += lst
        off.append(len(mem))
    return np.array(off, np.uint32), np.array(mem, np.uint32)
