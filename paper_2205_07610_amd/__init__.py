"""MI355X-native batched score-only pairwise alignment (Gotoh affine-gap DP).

The compute path is the C-ABI library ``libanyseq_mi.so`` (HIP for gfx950)
declared in ``include/anyseq_mi.h``; ``binding`` marshals arguments to it.
Importing this package loads nothing; ``binding.lib()`` loads the library and
raises if it has not been built.
"""
