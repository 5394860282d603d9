"""MI355X implementation of adaptive geometric multigrid with local smoothing
(arXiv:1904.03317): HIP library + thin Python binding."""
