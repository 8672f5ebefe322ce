"""The analysis routines of the package, for the tests."""
from paper_0904_0642_amd.analysis import autocorrelation, gaussian_difference_q, jackknife_mean, tau_int  # noqa: F401
