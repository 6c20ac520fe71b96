"""Oracle: plain, slow, obviously correct CPU implementations of what the
block-Wiedemann rank path computes.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check of the
package entry and the CPU baseline leg of the benchmark may import, call, link
or execute anything in it.  The GPU library never uses it, and it uses nothing
of the GPU library: the two share no code, headers, tables or helpers.

Contents (each function cites the passage of the paper it follows):

* ``ge``        rank over GF(p) by sparse and dense Gaussian elimination (the
                plain definition of the result, Section 2.5), Bareiss rank over Q.
* ``ge_rank.c`` the same sparse elimination in plain C, for mid-size inputs.
* ``sequence``  S_k = U^T B^k V with B = D_c A^T D A D_c (Sections 2.2, 2.3, 2.5).
* ``sigma``     Berlekamp-Massey, the iterative sigma-basis (M-Basis), the
                minimal matrix generator, its Popov form and the rank read-out
                deg det - codeg det (Sections 2.4, 2.5).
* ``splitmix``  the SplitMix64 generator from its published definition.

Parity status of every function is listed in its docstring; all are pinned by
the CPU tests (``-m "not gpu"``) against closed forms, brute force or textbook
routines.
"""
