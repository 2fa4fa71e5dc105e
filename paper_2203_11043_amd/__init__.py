"""MI355X-native hot path of the G-CoReCCD charge-transport simulator
(Avalos & Sofo Haro, arXiv 2203.11043).

Importing the package loads nothing; ``paper_2203_11043_amd.gccd`` binds the
HIP library ``libgccd.so`` and ``paper_2203_11043_amd.workloads`` draws seeded
synthetic inputs.
"""
