// gg_ttggg: diagram program not generated in this build
#include "../process.hpp"
namespace me { const ProcessDesc* process_gg_ttggg() { return nullptr; } }
