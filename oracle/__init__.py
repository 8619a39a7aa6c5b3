"""CPU FP64 oracle for the row-wise decomposed multi-dimensional FFT of
Duy & Ozaki, "A decomposition method with minimum communication amount for
parallelization of multi-dimensional FFTs".

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or link anything here;
the product library never does, and shares no code with it.

Modules
-------
dft        Eqs. (1)-(2): brute-force DFT, recursive mixed-radix FFT (C),
           axis-by-axis M-D FFT, error metrics.
decomp     Eqs. (4)-(19): levels, ranges, start/end points, owners point by
           point, communication amounts (readings R1 and R2), Eqs. (21)-(25).
orders     Eq. (20) / Table 1: valid transpose orders and their enumeration.
pipeline   Fig. 4 with explicit per-process arrays and an all-to-all.
rowsplit   the binary-exchange FFT of a row split over processes (level M),
           on explicit per-process blocks, with its exchanged points counted.

Parity status: every function is pinned by a test against values the paper
prints, closed forms, textbook identities or brute force.  The row-split
regime (level M) follows a stated reading in ``pipeline`` (a split row is
transformed whole); its values are pinned by the M-D DFT, its amounts by the
closed form at N_p = T (every point its own process).  The split row's own
exchange follows the binary-exchange reading, fitted to the 11.6 of Section
4 (the paper's algorithm for a split row is unknown); given that reading,
``decomp.split_row_volume`` is pinned against the points the executed
algorithm of ``rowsplit`` sends, and that algorithm against the DFT.
"""
