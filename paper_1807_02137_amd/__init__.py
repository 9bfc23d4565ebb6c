"""MI355X-native FAS multigrid with the jump-aware Hybrid Smoother 2 for the
selective level-set segmentation models of arXiv 1807.02137.

Importing the package loads nothing; ``paper_1807_02137_amd.mgseg`` loads the
HIP library (``lib/libmgseg.so``) on first use.
"""
