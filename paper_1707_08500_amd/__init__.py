"""MI355X-native local-FFT PSATD field push (Vincenti & Vay, Sec. 3).

Importing the package loads nothing; the HIP library is opened on first use
of :mod:`paper_1707_08500_amd.psatd`.
"""
