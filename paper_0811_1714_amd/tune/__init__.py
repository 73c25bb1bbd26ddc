"""Schedule tuning: timing datasets from the library's autotuner, training of the
schedule model on the GPU with the library's own MLP kernels, and evaluation."""
