"""Exact k-nearest-neighbour queries on embedded points and the majority vote
of the image-retrieval application (oracle, FP64).

Test infrastructure only: the library never imports this module.

Sec. 4.6 ("Approximate Nearest Neighbor Queries") runs a 10-nearest-neighbour
query in the database for each descriptor of a query photo and labels the
photo with the object that appears most often among the answers; accuracy
is the fraction of objects labelled correctly.  Sec. 4.7 ("Classification")
builds the k-nearest-neighbour graph (k = 30) of a point set.  Both are the
same operation: for every query q, the k database rows x with the smallest
||q - x||^2.

Readings:
* distances are squared Euclidean distances of the given FP32 rows, each
  difference and square in FP64 and the sum over coordinates in coordinate
  order;
* equal distances are ordered by the smaller database index, so the answer
  is unique;
* for the graph (queries = the database) a point is not its own neighbour:
  with exclude_self, query i skips database row i (other rows equal to it
  are ordinary neighbours at distance 0);
* a tied vote goes to the smallest object label (the paper draws at random
  among the tied objects; a fixed rule keeps the result reproducible).
"""
import numpy as np


def sq_dists(Q, D):
    """FP64 squared distances of every query row to every database row:
    sum_l (q_l - x_l)^2 by direct differences, summed in coordinate order."""
    Q = np.asarray(Q, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    out = np.zeros((Q.shape[0], D.shape[0]))
    for l in range(Q.shape[1]):
        diff = Q[:, l][:, None] - D[:, l][None, :]
        out += diff * diff
    return out


def knn(Q, D, k, exclude_self=False, block=256):
    """(idx, dist): for each query row, the indices of its k nearest database
    rows and their FP64 squared distances, ordered by (distance, index).
    Needs 1 <= k <= len(D) (len(D) - 1 with exclude_self)."""
    Q = np.asarray(Q)
    D = np.asarray(D)
    nd = D.shape[0]
    if not 1 <= k <= nd - (1 if exclude_self else 0):
        raise ValueError("k out of range")
    idx = np.empty((Q.shape[0], k), dtype=np.int64)
    dist = np.empty((Q.shape[0], k))
    for a in range(0, Q.shape[0], block):
        d2 = sq_dists(Q[a:a + block], D)
        if exclude_self:
            rows = np.arange(d2.shape[0])
            d2[rows, a + rows] = np.inf
        # lexsort: last key is primary -> distance first, then index
        order = np.lexsort((np.broadcast_to(np.arange(nd), d2.shape), d2), axis=1)[:, :k]
        idx[a:a + block] = order
        dist[a:a + block] = np.take_along_axis(d2, order, axis=1)
    return idx, dist


def vote(nn_idx, d_label, q_group, n_labels):
    """Majority vote per query group: every neighbour index of every query in
    a group adds one vote to its database label; the group's answer is the
    label with most votes, the smallest label among ties.  q_group[i] is the
    group of query i (groups 0 .. max)."""
    nn_idx = np.asarray(nn_idx)
    labels = np.asarray(d_label)[nn_idx]                 # nq x k
    groups = np.asarray(q_group)
    n_groups = int(groups.max()) + 1
    votes = np.zeros((n_groups, n_labels), dtype=np.int64)
    for i in range(labels.shape[0]):
        for lab in labels[i]:
            votes[groups[i], lab] += 1
    return votes.argmax(axis=1).astype(np.int32), votes     # argmax takes the first maximum


def accuracy(pred, truth):
    """Fraction of groups whose vote equals their true label."""
    return float(np.mean(np.asarray(pred) == np.asarray(truth)))
