"""In-order rank of a node of the complete binary tree stored in level order, by
counting subtree sizes on the walk to the root; used to check the Eytzinger
layout at sizes where the oracle's recursive fill is too slow."""


def subtree_size(i: int, n: int) -> int:
    """Nodes of the complete tree (level order, 1-based, n nodes) under node i."""
    size, lo, hi = 0, i, i
    while lo <= n:
        size += min(hi, n) - lo + 1
        lo, hi = 2 * lo, 2 * hi + 1
    return size


def inorder_rank(i: int, n: int) -> int:
    """In-order position (0-based) of node i: its left subtree, plus every ancestor
    that i lies to the right of, with that ancestor's left subtree."""
    rank = subtree_size(2 * i, n)
    while i > 1:
        parent = i // 2
        if i == 2 * parent + 1:
            rank += 1 + subtree_size(2 * parent, n)
        i = parent
    return rank
