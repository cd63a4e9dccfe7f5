"""Index maps of the paper's <L,S,C> schedules (Sec. 4), modelled in Python:
every output index is covered exactly once, for the paper's examples."""


def fp_indices(L, S, C, n_blocks):
    """Fully-Parallel: block k, thread t, loop l, element c -> one index; the
    tile is L*S*C and successive loop steps are S*C apart."""
    out = []
    tile = L * S * C
    for k in range(n_blocks):
        for t in range(S):
            for l in range(L):
                for c in range(C):
                    out.append(k * tile + l * S * C + t * C + c)
    return out


def gp_groups(L, S, C, n_groups):
    """Group-Parallel: C threads (C/S blocks) share a group; a block steps
    over groups by L*S/C."""
    blocks_per_group = C // S
    stride = L * S // C
    owner = {}
    for blk in range(L):
        g = blk // blocks_per_group
        while g < n_groups:
            owner.setdefault(g, set()).add(blk)
            g += stride
    return owner


def test_fp_example_2_2_4():
    idx = fp_indices(2, 2, 4, 3)
    assert sorted(idx) == list(range(3 * 16))
    # thread 0 of block 0 touches [0..4) then [8..12): stride S*C = 8
    assert fp_indices(2, 2, 4, 1)[:8] == [0, 1, 2, 3, 8, 9, 10, 11]


def test_gp_example_8_4_16():
    owner = gp_groups(8, 4, 16, 4)
    assert owner[0] == owner[2] == {0, 1, 2, 3}
    assert owner[1] == owner[3] == {4, 5, 6, 7}
