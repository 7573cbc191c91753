"""SVLF per-ray render path on MI355X (gfx950).

``svlf``      ctypes binding of libsvlf.so (the C-ABI in include/svlf.h)
``autograd``  torch.autograd.Function over svlf_render / svlf_render_backward
``train``     GPU training loop driven by svlf_train_step and svlf_adam_step
"""
