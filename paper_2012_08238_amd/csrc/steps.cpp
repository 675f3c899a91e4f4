// Stage plan of a set of signals launched together (see steps.hpp).
#include "steps.hpp"

#include <algorithm>
#include <set>

#include "kernels.hpp"

namespace sfft {

namespace {
constexpr uint32_t kFftLog2Max = 14;   // one-workgroup FFT sizes 2^1 .. 2^14
constexpr uint32_t kLargeLog2Min = 12; // two-pass FFT sizes 2^12 .. 2^18 (below 2^15 on request), three launches each
constexpr uint32_t kLargeLog2Max = 18;
constexpr uint32_t kLmaxCount = 4;     // lmax in {4, 8, 16, 32}
}  // namespace

size_t max_prefix_entries(size_t n) {
    // fold: at most one launch per distinct variant (<= n); fft: kFftLog2Max;
    // two-pass fft: 3 per size; comb prefilter: one per comb size (2^1 .. 2^14);
    // per round: vote 2 x kVoteKeys, phase decode 1, estimate kLmaxCount, top-K 1;
    // subtraction 1, reselection kFftLog2Max; residual and its sum 2; fused: one per L
    const size_t launches = n + kFftLog2Max + 3 * (kLargeLog2Max - kLargeLog2Min + 1) + kFftLog2Max +
                            2 * (2 * kVoteKeys + kLmaxCount + 2) + 1 + kFftLog2Max + 2 + kFusedMaxL;
    return launches * (n + 1);
}

void plan_steps(const std::vector<const Resolved*>& sig, std::vector<Step>* steps, std::vector<uint32_t>* prefix) {
    const size_t n = sig.size();
    // a fused signal takes part in its fused launch only, every other signal in the others
    auto add_step = [&](StepKind kind, uint32_t param, uint32_t lds, auto units_of) {
        const size_t off = prefix->size();
        uint32_t acc = 0;
        prefix->push_back(0);
        for (size_t i = 0; i < n; ++i) {
            if ((kind == kStepFused) == (sig[i]->fused != 0)) acc += units_of(*sig[i]);
            prefix->push_back(acc);
        }
        if (acc == 0) {
            prefix->resize(off);
            return;
        }
        steps->push_back(Step{kind, param, acc, lds, off});
    };
    auto max_of = [&](auto pred, auto field) {
        uint32_t v = 0;
        for (size_t i = 0; i < n; ++i)
            if (pred(*sig[i])) v = std::max(v, field(*sig[i]));
        return v;
    };
    for (uint32_t l = 1; l <= kFusedMaxL; ++l) {
        auto in_group = [&](const Resolved& R) { return R.fused && R.L == l; };
        add_step(kStepFused, l, max_of(in_group, [](const Resolved& R) { return R.fused_lds; }),
                 [&](const Resolved& R) { return in_group(R) ? 1u : 0u; });
    }
    std::set<uint32_t> variants;
    for (size_t i = 0; i < n; ++i)
        if (!sig[i]->fused) variants.insert(sig[i]->fold_variant);
    for (const uint32_t v : variants) {
        const uint32_t lds = max_of([&](const Resolved& R) { return R.fold_variant == v && R.mode == 1; },
                                    [](const Resolved& R) { return R.strip_lds; });
        add_step(kStepFold, v, lds, [&](const Resolved& R) { return R.fold_variant == v ? R.fold_units : 0u; });
    }
    for (uint32_t lb = 1; lb <= kFftLog2Max; ++lb)
        add_step(kStepFft, lb, 0, [&](const Resolved& R) { return !R.fft_mode && R.log2B == lb ? R.L : 0u; });
    for (uint32_t pass = 0; pass < 3; ++pass)
        for (uint32_t lb = kLargeLog2Min; lb <= kLargeLog2Max; ++lb)
            add_step(kStepFftLarge, lb | (pass << 8), 0, [&](const Resolved& R) {
                if (!R.fft_mode || R.log2B != lb) return 0u;
                return pass == 0 ? R.fft_p1_units : (pass == 1 ? R.fft_p2_units : R.L);
            });
    for (uint32_t lb = 1; lb <= kFftLog2Max; ++lb)
        add_step(kStepComb, lb, 0, [&](const Resolved& R) { return R.comb_loops && R.comb_log2b == lb ? R.comb_loops : 0u; });
    // location and estimation; the subtraction round repeats them for the signals that iterate
    for (uint32_t round = 0; round < 2; ++round) {
        auto active = [&](const Resolved& R) { return round == 0 || R.iterate; };
        if (round == 1) {
            add_step(kStepSub, 0, max_of(active, [](const Resolved& R) { return R.sub_lds; }),
                     [&](const Resolved& R) { return R.iterate ? R.L : 0u; });
            for (uint32_t lb = 1; lb <= kFftLog2Max; ++lb)
                add_step(kStepReselect, lb, 0, [&](const Resolved& R) { return R.iterate && R.log2B == lb ? R.L : 0u; });
        }
        for (uint32_t staged = 0; staged < 2; ++staged)
            for (uint32_t vk = 1; vk <= 32; ++vk) {
                if (vote_key(vk) != vk) continue;
                auto in_group = [&](const Resolved& R) {
                    return active(R) && !R.phase && (R.vote_lds > 0) == (staged == 1) && vote_key(R.L) == vk;
                };
                const uint32_t lds = max_of(in_group, [](const Resolved& R) { return R.vote_dyn_lds; });
                add_step(kStepVote, staged | (vk << 8) | (round << 16), lds,
                         [&](const Resolved& R) { return in_group(R) ? R.vote_units : 0u; });
            }
        add_step(kStepDecode, round, 0, [&](const Resolved& R) { return active(R) && R.phase ? R.vote_units : 0u; });
        for (uint32_t lm = 4; lm <= 32; lm <<= 1) {
            auto in_group = [&](const Resolved& R) { return active(R) && R.lmax == lm; };
            add_step(kStepEst, lm | (round << 8), 0, [&](const Resolved& R) { return in_group(R) ? R.est_units : 0u; });
        }
        add_step(kStepFin, round, max_of(active, [](const Resolved& R) { return R.fin_lds; }),
                 [&](const Resolved& R) { return active(R) && !R.est_only ? 1u : 0u; });
    }
    add_step(kStepRes, 0, max_of([](const Resolved& R) { return R.S > 0; }, [](const Resolved& R) { return R.resid_lds; }),
             [&](const Resolved& R) { return R.S ? R.resid_blocks : 0u; });
    add_step(kStepResSum, 0, 0, [&](const Resolved& R) { return R.S ? 1u : 0u; });
}

hipError_t issue_steps(const std::vector<Step>& steps, const SigDesc* d_descs, const IoDesc* d_ios,
                       const uint32_t* d_prefix, uint32_t n, uint32_t xcd_order, int part, hipStream_t s) {
    for (const Step& st : steps) {
        if (part >= 0 && (st.kind == kStepFold) != (part == 0)) continue;
        Launch a{};
        a.descs = d_descs;
        a.ios = d_ios;
        a.prefix = d_prefix + st.prefix_off;
        a.nsig = n;
        a.xcd_order = st.kind == kStepFold ? xcd_order : 0u;
        hipError_t e = hipSuccess;
        switch (st.kind) {
            case kStepFold: e = launch_fold(a, st.param, st.units, st.lds, s); break;
            case kStepFft: e = launch_fft_select(a, st.param, st.units, s); break;
            case kStepVote:
                e = launch_vote(a, (st.param >> 8) & 255u, st.units, st.lds, st.param & 1u, st.param >> 16, s);
                break;
            case kStepDecode: e = launch_decode(a, st.units, st.param, s); break;
            case kStepEst: e = launch_estimate(a, st.param & 255u, st.units, st.param >> 8, s); break;
            case kStepFin: e = launch_finalize(a, st.units, st.lds, st.param, s); break;
            case kStepSub: e = launch_subtract(a, st.units, st.lds, s); break;
            case kStepReselect: e = launch_reselect(a, st.param, st.units, s); break;
            case kStepRes: e = launch_residual(a, st.units, st.lds, s); break;
            case kStepResSum: e = launch_residual_sum(a, st.units, s); break;
            case kStepFftLarge: e = launch_fft_large(a, st.param & 255u, st.param >> 8, st.units, s); break;
            case kStepComb: e = launch_comb(a, st.param, st.units, s); break;
            case kStepFused: e = launch_fused(a, vote_key(st.param), st.units, st.lds, s); break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sfft
