"""Independent scipy.sparse view of a system in the compressed row format.

Written for the tests from the description of Section 3 of arXiv 2212.11675
(it shares no code with the oracle or the GPU library): the full matrix A has,
in row i, the 5 astrometric columns 5*star[i]+0..4, for each attitude axis a
the 4 columns 5*S + a*N_DFA + att[i] + 0..3, the 6 instrumental columns
5*S + 3*N_DFA + instr[i, :] and the global column 5*S + 3*N_DFA + N_instr.
"""
import numpy as np
import scipy.sparse as sp


def column_table(dims, star, att, instr):
    """[m, 24] int64 array of the column of every stored coefficient."""
    S, T, I = int(dims["n_stars"]), int(dims["n_dfa"]), int(dims["n_instr"])
    m = len(star)
    star = np.asarray(star, dtype=np.int64)
    att = np.asarray(att, dtype=np.int64)
    instr = np.asarray(instr, dtype=np.int64).reshape(m, 6)
    cols = np.empty((m, 24), dtype=np.int64)
    cols[:, 0:5] = 5 * star[:, None] + np.arange(5)[None, :]
    for a in range(3):
        cols[:, 5 + 4 * a: 9 + 4 * a] = 5 * S + a * T + att[:, None] + np.arange(4)[None, :]
    cols[:, 17:23] = 5 * S + 3 * T + instr
    cols[:, 23] = 5 * S + 3 * T + I
    return cols


def n_cols(dims):
    return 5 * int(dims["n_stars"]) + 3 * int(dims["n_dfa"]) + int(dims["n_instr"]) + 1


def csr(dims, vals, star, att, instr):
    m = len(star)
    cols = column_table(dims, star, att, instr)
    rows = np.repeat(np.arange(m), 24)
    A = sp.coo_matrix((np.asarray(vals, dtype=np.float64).ravel(), (rows, cols.ravel())),
                      shape=(m, n_cols(dims)))
    return A.tocsr()  # duplicates (if any) are summed, as the products do


def dense(dims, vals, star, att, instr):
    return csr(dims, vals, star, att, instr).toarray()
