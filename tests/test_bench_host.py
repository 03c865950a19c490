"""Host side of bench.py (no GPU): which kernel symbols the bench's labels
name, so that the roofline's traffic and time come from the kernel the step
runs."""
import bench


def test_adjoint_label_names_both_entry_points_at_its_stride():
    for name in ("k_adjoint", "k_adjoint_w2"):
        sym = f"void {name}<float, 6, 14, 4, false>(AdjArgs<float>)"
        assert bench.symbol_matches("adjoint", sym, 4)
        assert not bench.symbol_matches("adjoint", sym, 2)
    assert not bench.symbol_matches("adjoint", "void k_adjoint_pipe<float, 6, 14, 4>(AdjPipeArgs<float>)", 4)
    assert bench.symbol_matches("adjoint_pipe", "void k_adjoint_pipe<float, 6, 14, 4>(AdjPipeArgs<float>)", 4)


def test_sweep_labels_separate_the_checkpointing_sweep():
    ck = "void k_sweep<float, 6, 14, true, 4, false>(SweepArgs<float>)"
    plain = "void k_sweep<float, 6, 14, false, 4, false>(SweepArgs<float>)"
    assert bench.symbol_matches("sweep_ckpt", ck, 4) and not bench.symbol_matches("sweep_ckpt", ck, 2)
    assert not bench.symbol_matches("sweep_ckpt", plain, 4)
    assert bench.symbol_matches("sweep", plain, 4) and not bench.symbol_matches("sweep", ck, 4)
    assert not bench.symbol_matches("sweep", "void k_sweep_pipe<float, 6, 14, false, 4>(PipeArgs<float>)", 4)


def test_other_labels():
    assert bench.symbol_matches("gram", "void k_gram_direct<float>(GramArgs<float>)", 4)
    assert not bench.symbol_matches("gram", "void k_gram_pair<float, false>(GramArgs<float>)", 4)
    assert bench.symbol_matches("contract", "void k_contract<float, 8>(ContractArgs<float>)", 4)
    assert bench.symbol_matches("reduce", "void k_reduce_gram_y<float>(ReduceGramArgs<float>)", 4)
