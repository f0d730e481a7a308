"""MI355X-native CSF-MTTKRP and sparse CP-ALS (arXiv:1812.05961's hot path).

Import the binding explicitly: ``from paper_1812_05961_amd import cpd``.
"""
