"""Test helpers: moving oracle blocks into the library's block layout and back."""
from __future__ import annotations

import numpy as np


def pack_blocks(plan_host, blocks, ncols_of):
    """Flatten per-block dense matrices [m_j, K_j] into the column-major block layout."""
    blk_off = plan_host["blk_off"]
    out = np.zeros(max(int(blk_off[-1]), 1))
    for j, B in enumerate(blocks):
        out[blk_off[j]:blk_off[j + 1]] = np.asarray(B).ravel(order="F")
    return out


def pack_q(plan_host, facts, K):
    """Oracle Q_hat_j into the first r_j columns of each block's Q slot."""
    blk_off = plan_host["blk_off"]
    row_off = plan_host["row_off"]
    out = np.zeros(max(int(blk_off[-1]), 1))
    for j, f in enumerate(facts):
        m = int(row_off[j + 1] - row_off[j])
        slot = np.zeros((m, int(K[j])))
        slot[:, :f.rank] = f.Q
        out[blk_off[j]:blk_off[j + 1]] = slot.ravel(order="F")
    return out


def pack_r(plan_host, facts, K):
    rsq = plan_host["rsq_off"]
    out = np.zeros(max(int(rsq[-1]), 1))
    for j, f in enumerate(facts):
        slot = np.zeros((int(K[j]), int(K[j])))
        slot[:f.rank, :f.rank] = f.R
        out[rsq[j]:rsq[j + 1]] = slot.ravel(order="F")
    return out


def pack_kept(plan_host, facts, K):
    fo = plan_host["feat_off"]
    out = np.full(max(int(fo[-1]), 1), -1, dtype=np.int32)
    for j, f in enumerate(facts):
        out[fo[j]:fo[j] + f.rank] = f.kept
    return out


def pack_y(feat_off, facts, y_compact):
    out = np.zeros(max(int(feat_off[-1]), 1))
    pos = 0
    for j, f in enumerate(facts):
        out[feat_off[j]:feat_off[j] + f.rank] = y_compact[pos:pos + f.rank]
        pos += f.rank
    return out


def unpack_block(flat, plan_host, j, K):
    blk_off = plan_host["blk_off"]
    row_off = plan_host["row_off"]
    m = int(row_off[j + 1] - row_off[j])
    return np.asarray(flat[blk_off[j]:blk_off[j + 1]]).reshape((m, int(K[j])), order="F")


def unpack_r(flat, plan_host, j, K, r):
    rsq = plan_host["rsq_off"]
    return np.asarray(flat[rsq[j]:rsq[j + 1]]).reshape((int(K[j]), int(K[j])), order="F")[:r, :r]


def oracle_rows(plan_host):
    ro = plan_host["row_off"]
    return [plan_host["rows"][ro[j]:ro[j + 1]] for j in range(len(ro) - 1)]
